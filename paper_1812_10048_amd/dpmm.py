"""ctypes binding of libdpmm (include/dpmm.h): argument marshalling only.

Every function here has the name of the C entry point it calls and raises
``DpmmError`` with the library's message when the status is not DPMM_OK.
There is no fallback: if ``libdpmm.so`` has not been built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpmm.so")

DPMM_OK = 0
DPMM_ERR_ARG = -1
DPMM_ERR_HIP = -2
DPMM_ERR_NOMEM = -3
DPMM_ERR_STATE = -4
DPMM_ERR_UNSUPPORTED = -5
DPMM_ERR_DATA = -6
STATUS_NAMES = {0: "DPMM_OK", -1: "DPMM_ERR_ARG", -2: "DPMM_ERR_HIP", -3: "DPMM_ERR_NOMEM",
                -4: "DPMM_ERR_STATE", -5: "DPMM_ERR_UNSUPPORTED", -6: "DPMM_ERR_DATA"}

DPMM_FP64, DPMM_FP32, DPMM_SPLIT_BF16 = 0, 1, 2
PRECISIONS = {"fp64": DPMM_FP64, "fp32": DPMM_FP32, "split_bf16": DPMM_SPLIT_BF16}
FLAG_SPLIT_Q = 1     # DPMM_FLAG_SPLIT_Q
FLAG_NEW_CLUSTER = 2     # DPMM_FLAG_NEW_CLUSTER
FLAG_RANDOM_SPLIT = 4     # DPMM_FLAG_RANDOM_SPLIT
FLAGS_PAPER = FLAG_SPLIT_Q | FLAG_NEW_CLUSTER | FLAG_RANDOM_SPLIT     # DPMM_FLAGS_PAPER


class DpmmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class dpmm_csr(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_genes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class dpmm_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("beta_per_gene", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("k_init", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32), ("refine_tol", ctypes.c_double)]


class dpmm_stats_out(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("K", ctypes.c_int32), ("last_pass", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("sm_calls", ctypes.c_int64),
                ("splits_proposed", ctypes.c_int64), ("splits_accepted", ctypes.c_int64),
                ("merges_proposed", ctypes.c_int64), ("merges_accepted", ctypes.c_int64),
                ("kmax_skips", ctypes.c_int64), ("refined", ctypes.c_int64), ("gamma_caps", ctypes.c_int64),
                ("evals", ctypes.c_int64), ("near_tie", ctypes.c_int64), ("log_joint", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# DPMM_STAGE_* of include/dpmm.h, in order
STAGES = ["redraw", "assign", "refine", "subcluster", "compact", "split_merge", "eb", "layout"]


_P = ctypes.c_void_p
_S = ctypes.c_int
_SIGNATURES = {
    "dpmm_last_error": ([], ctypes.c_char_p),
    "dpmm_workspace_size": ([ctypes.POINTER(dpmm_csr), ctypes.POINTER(dpmm_params), ctypes.POINTER(ctypes.c_size_t)], _S),
    "dpmm_init": ([ctypes.POINTER(dpmm_csr), ctypes.POINTER(dpmm_params), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], _S),
    "dpmm_init_static": ([ctypes.POINTER(dpmm_csr), ctypes.POINTER(dpmm_params), _P, ctypes.POINTER(_P)], _S),
    "dpmm_destroy": ([_P], _S),
    "dpmm_sweep": ([_P, ctypes.c_int32], _S),
    "dpmm_split_merge": ([_P], _S),
    "dpmm_eb_update": ([_P], _S),
    "dpmm_stats": ([_P, ctypes.POINTER(dpmm_stats_out), _P, _P], _S),
    "dpmm_get_labels": ([_P, _P, _P], _S),
    "dpmm_set_state": ([_P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P], _S),
    "dpmm_get_reset_flags": ([_P, _P], _S),
    "dpmm_get_params": ([_P, _P, _P], _S),
    "dpmm_get_beta": ([_P, _P], _S),
    "dpmm_set_beta": ([_P, _P], _S),
    "dpmm_get_hastings": ([_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _P, _P], _S),
    "dpmm_set_debug_scores": ([_P, _P, ctypes.c_int32, ctypes.c_int32], _S),
    "dpmm_dump_scores": ([_P, _P, ctypes.c_int32, _P], _S),
    "dpmm_get_split_tables": ([_P, _P, _P], _S),
    "dpmm_timing_enable": ([_P, ctypes.c_int32], _S),
    "dpmm_timing_read": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], _S),
    "dpmm_timing_stages": ([_P, _P, _P], _S),
    "dpmm_dm_logmarginal": ([_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P], _S),
    "dpmm_dm_grad": ([_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P], _S),
    "dpmm_gene_moments": ([ctypes.POINTER(dpmm_csr), _P, _P, _P], _S),
    "dpmm_filter_genes": ([ctypes.POINTER(dpmm_csr), _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64), _P], _S),
    "dpmm_top_genes": ([_P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P, _P], _S),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libdpmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1812_10048_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def dpmm_last_error() -> str:
    return lib().dpmm_last_error().decode()


def _check(status: int) -> None:
    if status != DPMM_OK:
        raise DpmmError(status, dpmm_last_error())


def dpmm_workspace_size(csr: dpmm_csr, params: dpmm_params) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().dpmm_workspace_size(ctypes.byref(csr), ctypes.byref(params), ctypes.byref(out)))
    return out.value


def dpmm_init(csr: dpmm_csr, params: dpmm_params, workspace: int, workspace_bytes: int, stream: int) -> int:
    ctx = _P(0)
    _check(lib().dpmm_init(ctypes.byref(csr), ctypes.byref(params), workspace, workspace_bytes, stream,
                           ctypes.byref(ctx)))
    return ctx.value


def dpmm_init_static(csr: dpmm_csr, params: dpmm_params, stream: int) -> int:
    ctx = _P(0)
    _check(lib().dpmm_init_static(ctypes.byref(csr), ctypes.byref(params), stream, ctypes.byref(ctx)))
    return ctx.value


def dpmm_destroy(ctx: int) -> None:
    _check(lib().dpmm_destroy(ctx))


def dpmm_sweep(ctx: int, n_sweeps: int) -> None:
    _check(lib().dpmm_sweep(ctx, n_sweeps))


def dpmm_split_merge(ctx: int) -> None:
    _check(lib().dpmm_split_merge(ctx))


def dpmm_eb_update(ctx: int) -> None:
    _check(lib().dpmm_eb_update(ctx))


def dpmm_stats(ctx: int, nsub_host: int = 0, ssub_dev: int = 0) -> dpmm_stats_out:
    out = dpmm_stats_out()
    _check(lib().dpmm_stats(ctx, ctypes.byref(out), nsub_host or None, ssub_dev or None))
    return out


def dpmm_get_labels(ctx: int, c_dev: int, cs_dev: int) -> None:
    _check(lib().dpmm_get_labels(ctx, c_dev, cs_dev))


def dpmm_set_state(ctx: int, step: int, K: int, c_dev: int, cs_dev: int, reset_host: int) -> None:
    _check(lib().dpmm_set_state(ctx, step, K, c_dev, cs_dev, reset_host))


def dpmm_get_reset_flags(ctx: int, reset_host: int) -> None:
    _check(lib().dpmm_get_reset_flags(ctx, reset_host))


def dpmm_get_params(ctx: int, logpi_dev: int, logtheta_dev: int) -> None:
    _check(lib().dpmm_get_params(ctx, logpi_dev or None, logtheta_dev or None))


def dpmm_get_beta(ctx: int, beta_dev: int) -> None:
    _check(lib().dpmm_get_beta(ctx, beta_dev))


def dpmm_set_beta(ctx: int, beta_dev: int) -> None:
    _check(lib().dpmm_set_beta(ctx, beta_dev))


def dpmm_get_hastings(ctx: int, logr_host: int = 0, accept_host: int = 0):
    p = ctypes.c_int32(0)
    n = ctypes.c_int32(0)
    _check(lib().dpmm_get_hastings(ctx, ctypes.byref(p), ctypes.byref(n), logr_host or None, accept_host or None))
    return p.value, n.value


def dpmm_set_debug_scores(ctx: int, scores_dev: int, k_cap: int, fp64: bool = False) -> None:
    _check(lib().dpmm_set_debug_scores(ctx, scores_dev or None, k_cap, 1 if fp64 else 0))


def dpmm_dump_scores(ctx: int, cells_dev: int, m: int, out_dev: int) -> None:
    _check(lib().dpmm_dump_scores(ctx, cells_dev or None, m, out_dev or None))


def dpmm_get_split_tables(ctx: int, hi_dev: int, lo_dev: int) -> None:
    _check(lib().dpmm_get_split_tables(ctx, hi_dev, lo_dev))


def dpmm_timing_enable(ctx: int, enable: bool) -> None:
    _check(lib().dpmm_timing_enable(ctx, 1 if enable else 0))


def dpmm_timing_stages(ctx: int) -> dict:
    """{stage: (milliseconds, intervals)} since the last read."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    _check(lib().dpmm_timing_stages(ctx, ms, n))
    return {name: (ms[j], n[j]) for j, name in enumerate(STAGES)}


def dpmm_timing_read(ctx: int):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().dpmm_timing_read(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def dpmm_dm_logmarginal(s_dev: int, J: int, G: int, beta_dev: int, out_dev: int, stream: int) -> None:
    _check(lib().dpmm_dm_logmarginal(s_dev, J, G, beta_dev, out_dev, stream))


def dpmm_dm_grad(s_dev: int, J: int, G: int, beta_dev: int, g_dev: int, grad_dev: int, stream: int) -> None:
    _check(lib().dpmm_dm_grad(s_dev, J, G, beta_dev, g_dev, grad_dev, stream))


def dpmm_gene_moments(csr: dpmm_csr, sum_dev: int, sumsq_dev: int, stream: int) -> None:
    _check(lib().dpmm_gene_moments(ctypes.byref(csr), sum_dev, sumsq_dev, stream))


def dpmm_top_genes(sum_dev: int, sumsq_dev: int, n_genes: int, n_cells: int, k: int, map_dev: int, std_dev,
                   stream: int) -> None:
    _check(lib().dpmm_top_genes(sum_dev, sumsq_dev, int(n_genes), int(n_cells), int(k), map_dev, std_dev, stream))


def dpmm_filter_genes(csr: dpmm_csr, map_dev: int, row_ptr_out: int, col_out, val_out, stream: int) -> int:
    """First call with col_out = None returns the new nnz; the second fills."""
    n = ctypes.c_int64(0)
    _check(lib().dpmm_filter_genes(ctypes.byref(csr), map_dev, row_ptr_out, col_out, val_out, ctypes.byref(n), stream))
    return int(n.value)
