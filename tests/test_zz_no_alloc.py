"""dpmm_init_static, the entry point that allocates nothing, against dpmm_init.

The static context takes its workspace from the library's per-device static
array instead of a caller buffer, and sizes its launches for k_max instead of
a host hint.  Two calls in a row (2,000 cells, then 800 cells of a different
matrix, so the second finds the first one's contents in the array): each runs
ten iterations beside a dpmm_init context on the same data and seed, and the
labels, statistics and Hastings ratios are compared after every step,
bit-exact (both run the same kernels on the same inputs).  A matrix larger
than the static workspace and a second static context on the same GPU are
refused with clear errors.
"""
import numpy as np
import pytest
import torch

from lockstep import say
from paper_1812_10048_amd import dpmm as C
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu


def _same(a, b, what):
    ca, csa = a.labels()
    cb, csb = b.labels()
    assert torch.equal(ca, cb) and torch.equal(csa, csb), what
    sa, sb = a.stats(with_tables=True), b.stats(with_tables=True)
    assert sa["K"] == sb["K"], what
    assert np.array_equal(sa["nsub"], sb["nsub"]), what
    assert torch.equal(sa["ssub"], sb["ssub"]), what


@pytest.mark.parametrize("precision", ["split_bf16", "fp32"])
def test_static_workspace_matches_dpmm_init(precision):
    for n_cells, seed in ((2000, 0), (800, 3)):
        say("no-alloc", precision, n_cells)
        d = synth.generate("c1", seed=seed, n_cells=n_cells)
        kw = dict(alpha=1.0, beta=1.0, seed=seed + 7, k_max=32, k_init=1, precision=precision)
        st = Sampler(d.row_ptr, d.col, d.val, d.n_genes, static_workspace=True, **kw)
        assert st._ws is None
        ref = Sampler(d.row_ptr, d.col, d.val, d.n_genes, **kw)
        _same(st, ref, "init")
        for it in range(10):
            st.sweep(1)
            ref.sweep(1)
            _same(st, ref, f"sweep {it}")
            st.split_merge()
            ref.split_merge()
            pa, la, aa = st.hastings()
            pb, lb, ab = ref.hastings()
            assert pa == pb and np.array_equal(la, lb, equal_nan=True) and np.array_equal(aa, ab)
            _same(st, ref, f"split/merge {it}")
        assert st.K >= 2
        say("no-alloc", precision, n_cells, "K", st.K)
        st.close()
        ref.close()


def test_static_workspace_limits():
    say("no-alloc limits")
    d = synth.generate("c1", seed=1, n_cells=500)
    a = Sampler(d.row_ptr, d.col, d.val, d.n_genes, static_workspace=True, k_max=16)
    with pytest.raises(C.DpmmError) as e:
        Sampler(d.row_ptr, d.col, d.val, d.n_genes, static_workspace=True, k_max=16)
    assert e.value.status == C.DPMM_ERR_STATE
    a.close()
    # once released, the storage can be taken again
    b = Sampler(d.row_ptr, d.col, d.val, d.n_genes, static_workspace=True, k_max=16)
    b.iterate(2)
    b.close()
    big = synth.generate("c2", seed=0, n_cells=60000)
    with pytest.raises(C.DpmmError) as e:
        Sampler(big.row_ptr, big.col, big.val, big.n_genes, static_workspace=True, precision="split_bf16")
    assert e.value.status == C.DPMM_ERR_NOMEM
