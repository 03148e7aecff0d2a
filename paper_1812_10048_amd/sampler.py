"""Python face of libdpmm: ``Sampler``, ``DMLogMarginal`` and ``eb_update_beta``.

Torch supplies device memory (the workspace and the arrays handed to the C
ABI) and the stream; every step of the sampler runs in the library's HIP
kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dpmm as C


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype) -> torch.Tensor:
    return t.to(device="cuda", dtype=dtype).contiguous()


class Sampler:
    """Sub-cluster split/merge sampler over a cell-major CSR count matrix.

    Parameters follow ``dpmm_params`` in include/dpmm.h.  ``beta`` is a float
    or a length-G tensor of per-gene concentrations.  ``precision`` is one of
    "fp64", "fp32", "split_bf16".  ``split_q`` sets DPMM_FLAG_SPLIT_Q (the
    split ratio carries the proposal term of Section 2.3); ``new_cluster``
    sets DPMM_FLAG_NEW_CLUSTER (the Gibbs step runs over K + 1 clusters,
    eq. 4); ``random_split`` sets DPMM_FLAG_RANDOM_SPLIT (a third pass of
    random splits, chain B of Section 2.4).  All three are on by default
    (DPMM_FLAGS_PAPER, the moves as the paper states them); all off gives the
    collapsed split ratio alone.  ``static_workspace`` creates the context
    with dpmm_init_static (no allocation; small matrices only, one such
    sampler per GPU at a time).
    """

    def __init__(self, row_ptr, col, val, n_genes: int, *, alpha: float = 1.0, beta=1.0, seed: int = 0,
                 k_init: int = 1, k_max: int = 128, precision: str = "fp32", refine_tol: float = -1.0,
                 split_q: bool = True, new_cluster: bool = True, random_split: bool = True,
                 static_workspace: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libdpmm needs a GPU")
        rp = _dev(torch.as_tensor(row_ptr), torch.int64)
        cl = _dev(torch.as_tensor(col), torch.int32)
        vl = _dev(torch.as_tensor(val), torch.int32)
        self.N = rp.numel() - 1
        self.G = int(n_genes)
        self.k_max = int(k_max)
        self.precision = precision
        csr = C.dpmm_csr(self.N, self.G, 0, cl.numel(), rp.data_ptr(), cl.data_ptr() if cl.numel() else None,
                         vl.data_ptr() if vl.numel() else None)
        beta_t = None
        if isinstance(beta, (int, float)):
            beta_scalar = float(beta)
        else:
            beta_t = _dev(torch.as_tensor(beta), torch.float64)
            beta_scalar = 0.0
        params = C.dpmm_params(float(alpha), beta_scalar, beta_t.data_ptr() if beta_t is not None else None,
                               int(seed) & 0xFFFFFFFFFFFFFFFF, int(k_init), self.k_max, C.PRECISIONS[precision],
                               (C.FLAG_SPLIT_Q if split_q else 0) | (C.FLAG_NEW_CLUSTER if new_cluster else 0) |
                               (C.FLAG_RANDOM_SPLIT if random_split else 0), float(refine_tol))
        if static_workspace:
            # the library's static per-device workspace (dpmm_init_static)
            self._ws = None
            self._ctx = C.dpmm_init_static(csr, params, _stream())
        else:
            nbytes = C.dpmm_workspace_size(csr, params)
            # 256-byte alignment inside a slightly larger buffer
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            off = (-base) % 256
            self._ctx = C.dpmm_init(csr, params, base + off, nbytes, _stream())
        self._dbg = None

    # -- lifetime ----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            C.dpmm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- moves ---------------------------------------------------------------
    def sweep(self, n: int = 1) -> None:
        C.dpmm_sweep(self._ctx, int(n))

    def split_merge(self) -> None:
        C.dpmm_split_merge(self._ctx)

    def eb_update(self) -> None:
        C.dpmm_eb_update(self._ctx)

    def iterate(self, n: int = 1, eb_every: int = 0) -> None:
        """n iterations of (sweep, split/merge), with an empirical-Bayes step
        after every ``eb_every``-th iteration when > 0."""
        for it in range(n):
            self.sweep(1)
            self.split_merge()
            if eb_every and (it + 1) % eb_every == 0:
                self.eb_update()

    # -- state ----------------------------------------------------------------
    def stats(self, with_tables: bool = False) -> dict:
        nsub = np.zeros(2 * self.k_max, dtype=np.int64)
        ssub = torch.zeros(2 * self.k_max * self.G, dtype=torch.int64, device="cuda") if with_tables else None
        out = C.dpmm_stats(self._ctx, nsub.ctypes.data, ssub.data_ptr() if with_tables else 0).as_dict()
        K = out["K"]
        out["nsub"] = nsub[: 2 * K].copy()
        if with_tables:
            out["ssub"] = ssub[: 2 * K * self.G].view(2 * K, self.G)
        return out

    @property
    def K(self) -> int:
        return C.dpmm_stats(self._ctx).K

    def labels(self):
        c = torch.empty(self.N, dtype=torch.int32, device="cuda")
        cs = torch.empty(self.N, dtype=torch.uint8, device="cuda")
        C.dpmm_get_labels(self._ctx, c.data_ptr(), cs.data_ptr())
        return c, cs

    def reset_flags(self) -> np.ndarray:
        r = np.zeros(self.k_max, dtype=np.uint8)
        C.dpmm_get_reset_flags(self._ctx, r.ctypes.data)
        return r[: self.K].copy()

    def snapshot(self) -> dict:
        """Everything a resumed chain needs: (step, K, c, cbar, reset, beta)."""
        st = self.stats()
        c, cs = self.labels()
        return dict(step=st["step"], K=st["K"], c=c, cs=cs, reset=self.reset_flags(), beta=self.beta)

    def set_state(self, step: int, K: int, c, cs, reset) -> None:
        c = _dev(torch.as_tensor(c), torch.int32)
        cs = _dev(torch.as_tensor(cs), torch.uint8)
        r = np.zeros(max(1, int(K)), dtype=np.uint8)
        r[: len(reset)] = np.asarray(reset, dtype=np.uint8)[: int(K)]
        C.dpmm_set_state(self._ctx, int(step), int(K), c.data_ptr(), cs.data_ptr(), r.ctypes.data)

    def params(self):
        """(log pi [k_max], log theta [3 k_max, G]) of the last redraw, FP64."""
        lp = torch.empty(self.k_max, dtype=torch.float64, device="cuda")
        lt = torch.empty(3 * self.k_max, self.G, dtype=torch.float64, device="cuda")
        C.dpmm_get_params(self._ctx, lp.data_ptr(), lt.data_ptr())
        return lp, lt

    @property
    def beta(self) -> torch.Tensor:
        b = torch.empty(self.G, dtype=torch.float64, device="cuda")
        C.dpmm_get_beta(self._ctx, b.data_ptr())
        return b

    @beta.setter
    def beta(self, value) -> None:
        b = _dev(torch.as_tensor(value), torch.float64)
        C.dpmm_set_beta(self._ctx, b.data_ptr())

    def hastings(self):
        """(pass, log R [n], accepted [n]) of the last split/merge call."""
        cap = self.k_max + self.k_max * (self.k_max - 1) // 2
        logr = np.zeros(cap, dtype=np.float64)
        acc = np.zeros(cap, dtype=np.uint8)
        p, n = C.dpmm_get_hastings(self._ctx, logr.ctypes.data, acc.ctypes.data)
        return p, logr[:n].copy(), acc[:n].copy()

    def debug_scores(self, k_cap: int | None, fp64: bool = False):
        """Start (k_cap given) or stop (None) the per-cell score dump of the
        sweeps' own arithmetic; returns the [N, k_cap + 2] buffer (FP32, or
        FP64 with ``fp64``) the next sweeps write into."""
        if k_cap is None:
            C.dpmm_set_debug_scores(self._ctx, 0, 0)
            self._dbg = None
            return None
        dt = torch.float64 if fp64 else torch.float32
        self._dbg = torch.full((self.N, k_cap + 2), float("nan"), dtype=dt, device="cuda")
        C.dpmm_set_debug_scores(self._ctx, self._dbg.data_ptr(), int(k_cap), fp64)
        return self._dbg

    def dump_scores(self, cells) -> torch.Tensor:
        """FP64 [m, K + 2] log-likelihoods of the listed cells against the last
        redraw's parameters: K clusters, then the two sub-clusters of each
        cell's current cluster."""
        cl = _dev(torch.as_tensor(cells), torch.int32)
        K = self.K
        out = torch.empty(cl.numel(), K + 2, dtype=torch.float64, device="cuda")
        C.dpmm_dump_scores(self._ctx, cl.data_ptr(), cl.numel(), out.data_ptr())
        return out

    def split_tables(self):
        K = self.K
        hi = torch.empty(K, self.G, dtype=torch.int16, device="cuda")
        lo = torch.empty(K, self.G, dtype=torch.int16, device="cuda")
        C.dpmm_get_split_tables(self._ctx, hi.data_ptr(), lo.data_ptr())
        return hi, lo

    def timing(self, enable: bool) -> None:
        C.dpmm_timing_enable(self._ctx, enable)

    def timing_read(self):
        return C.dpmm_timing_read(self._ctx)

    def timing_stages(self) -> dict:
        return C.dpmm_timing_stages(self._ctx)


class DMLogMarginal(torch.autograd.Function):
    """out[j] = log Dirichlet-multinomial marginal of count vector s[j] under
    concentration beta (per gene); differentiable in beta."""

    @staticmethod
    def forward(ctx, beta: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
        beta_c = beta.detach().to(dtype=torch.float64).contiguous()
        s_c = s.to(dtype=torch.int64).contiguous()
        J, G = s_c.shape
        out = torch.empty(J, dtype=torch.float64, device=beta.device)
        C.dpmm_dm_logmarginal(s_c.data_ptr(), J, G, beta_c.data_ptr(), out.data_ptr(), _stream())
        ctx.save_for_backward(beta_c, s_c)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        beta_c, s_c = ctx.saved_tensors
        J, G = s_c.shape
        g = grad_out.to(dtype=torch.float64).contiguous()
        grad = torch.empty(G, dtype=torch.float64, device=beta_c.device)
        C.dpmm_dm_grad(s_c.data_ptr(), J, G, beta_c.data_ptr(), g.data_ptr(), grad.data_ptr(), _stream())
        return grad, None


def eb_update_beta(sampler: Sampler) -> torch.Tensor:
    """One empirical-Bayes fixed-point step of the sampler's per-gene beta."""
    sampler.eb_update()
    return sampler.beta
