"""The C-ABI library loads and exports every entry point include/dpmm.h
declares; host-only argument validation (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1812_10048_amd import dpmm as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dpmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpmm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dpmm_init", "dpmm_sweep", "dpmm_split_merge", "dpmm_stats", "dpmm_dm_grad", "dpmm_eb_update"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(C.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps each of them
    assert set(_declared()) <= set(C._SIGNATURES)


def _csr(N=10, G=5, nnz=20):
    return C.dpmm_csr(N, G, 0, nnz, 1, 1, 1)


def _params(**kw):
    p = dict(alpha=1.0, beta=1.0, beta_per_gene=None, seed=0, k_init=1, k_max=16, precision=C.DPMM_FP32,
             flags=0, refine_tol=-1.0)
    p.update(kw)
    return C.dpmm_params(**p)


def test_workspace_size_is_a_host_function():
    small = C.dpmm_workspace_size(_csr(), _params())
    big = C.dpmm_workspace_size(_csr(N=1000, G=500, nnz=100000), _params(k_max=64))
    assert 0 < small < big
    assert small % 256 == 0


@pytest.mark.parametrize("bad", [
    dict(csr=dict(N=0)), dict(csr=dict(G=0)), dict(csr=dict(G=70000)), dict(csr=dict(nnz=-1)),
    dict(params=dict(alpha=0.0)), dict(params=dict(beta=-1.0)), dict(params=dict(k_max=0)),
    dict(params=dict(k_max=2000)), dict(params=dict(k_init=0)), dict(params=dict(k_init=17)),
    dict(params=dict(precision=7)), dict(params=dict(flags=8)),
])
def test_invalid_arguments_are_rejected_with_a_message(bad):
    csr = _csr(**bad.get("csr", {}))
    params = _params(**bad.get("params", {}))
    with pytest.raises(C.DpmmError) as e:
        C.dpmm_workspace_size(csr, params)
    assert e.value.status == C.DPMM_ERR_ARG
    assert C.dpmm_last_error()


def test_null_context_is_an_error_not_a_crash():
    with pytest.raises(C.DpmmError) as e:
        C.dpmm_sweep(None, 1)
    assert e.value.status == C.DPMM_ERR_ARG
