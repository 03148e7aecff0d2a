"""The beta gradient and the empirical-Bayes step on the GPU at the
100,000 x 2,000 scale (12 power-law clusters, per-gene beta starting at 0.5,
an EB step every 10 sweeps), through the C ABI.

  * every EB step: beta on the GPU within 1e-9 relative of the oracle's step
    taken from the same labels;
  * at the end: the gradient of sum_j g_j logDM(s_j; beta) over the 3K count
    vectors (clusters, then sub-clusters) within 1e-9 of the FP64 oracle, and
    within 1e-6 of central differences evaluated in mpmath (h = 1e-6 min(1,
    beta_u), 40 digits: EB may drive a beta_u to its 1e-6 floor) on 50 genes
    chosen with Philox draws.
"""
import sys

import mpmath
import numpy as np
import pytest
import torch

import oracle
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import DMLogMarginal, Sampler

pytestmark = pytest.mark.gpu

mpmath.mp.dps = 40
H = mpmath.mpf("1e-6")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _philox_genes(G, n, key=0x5EED):
    genes, i = [], 0
    while len(genes) < n:
        g = int(oracle.philox4x32_10(key, [i, 0, 0, 0])[0]) % G
        if g not in genes:
            genes.append(g)
        i += 1
    return genes


def _fd(s, beta, g, u):
    S = s.sum(axis=1)
    B0 = mpmath.fsum(mpmath.mpf(float(b)) for b in beta)
    bu = mpmath.mpf(float(beta[u]))
    h = H * min(1, bu)          # beta_u may sit at the 1e-6 floor of the EB clamp

    def f(delta):
        B, b = B0 + delta, bu + delta
        return mpmath.fsum(mpmath.mpf(float(gj)) * (mpmath.loggamma(B) - mpmath.loggamma(B + int(Sj)) +
                                                     mpmath.loggamma(b + int(sj[u])) - mpmath.loggamma(b))
                           for sj, Sj, gj in zip(s, S, g))

    return float((f(h) - f(-h)) / (2 * h))


def test_c4_beta_gradient_and_empirical_bayes():
    _say("c4 gradient: generate")
    d = synth.generate("c4", seed=0, device="cuda")
    G, K0 = d.n_genes, d.n_true
    rp, col, val = d.host_arrays()
    kw = dict(alpha=1.0, seed=11, k_max=64)
    s = Sampler(d.row_ptr, d.col, d.val, G, beta=torch.full((G,), 0.5, dtype=torch.float64), k_init=1,
                precision="split_bf16", **kw)
    rng = np.random.default_rng(5)
    s.set_state(0, K0, torch.from_numpy(d.z), torch.from_numpy(rng.integers(0, 2, size=d.n_cells)),
                np.ones(K0, dtype=np.uint8))
    for it in range(20):
        s.sweep(1)
        s.split_merge()
        if it % 10 == 9:
            _say(f"c4 gradient: EB step after sweep {it + 1}")
            snap = s.snapshot()
            o = oracle.Oracle(rp, col, val, G, beta=snap["beta"].cpu().numpy(), init=False, **kw)
            o.set_state(snap["step"], snap["K"], snap["c"].cpu().numpy(), snap["cs"].cpu().numpy(),
                        np.asarray(snap["reset"]))
            o.eb_update()
            s.eb_update()
            b = s.beta.cpu().numpy()
            assert np.all(np.abs(b - o.beta) <= 1e-9 * np.abs(o.beta)), np.max(np.abs(b - o.beta) / o.beta)
    st = s.stats(with_tables=True)
    K = st["K"]
    ssub = st["ssub"]
    sv = torch.cat([ssub[0::2] + ssub[1::2], ssub]).contiguous()
    s_np = sv.cpu().numpy()
    beta_np = s.beta.cpu().numpy()
    genes = _philox_genes(G, 50)
    for name, g_np in (("all", np.ones(3 * K)), ("clusters", np.r_[np.ones(K), np.zeros(2 * K)])):
        _say(f"c4 gradient: weights {name}, K = {K}")
        beta = s.beta.clone().requires_grad_(True)
        out = DMLogMarginal.apply(beta, sv)
        (out * torch.tensor(g_np, device="cuda")).sum().backward()
        got = beta.grad.cpu().numpy()
        gref = oracle.dm_grad(s_np, beta_np, g_np)
        assert np.all(np.abs(got - gref) <= 1e-9 * np.maximum(1.0, np.abs(gref)))
        for u in genes:
            ref = _fd(s_np, beta_np, g_np, u)
            assert abs(got[u] - ref) <= 1e-6 * max(1.0, abs(ref)), (name, u, got[u], ref)
