"""The certified rounding bound of the split-BF16 scores on adversarial data,
on the GPU through the C ABI.

Every cell has a non-zero count for every gene (rows as long as the matrix is
wide), counts above 255 on the top genes (so those entries go to the FP32 tail
of the cluster-sorted copy), and the new cluster of the Gibbs step over K + 1
(eq. 4) has parameters drawn from the prior, whose log theta reach far below
the posterior clusters'.  All terms x log theta have the same sign, so the
rounding errors cannot cancel by sign.  With G = 512 every gene fits the dense
chunks (the matrix cores do nearly all the work); with G = 2000 three quarters
of each row is tail.  For every cell i and cluster k the kernel's own score
must satisfy
    |S_ik - S_ik(FP64)| <= (2^-17 + (2 n_i + 8) 2^-23) 1.01 (|S_ik| + 20) + 1e-5,
the bound the kernel certifies its decisions with (log pi = 0 here), where n_i
is the cell's number of non-zero counts and S(FP64) comes from the oracle with
the same parameters.
"""
import numpy as np
import pytest
import torch

import oracle
from lockstep import report, say
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu


def adversarial(n_cells: int, n_genes: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    rate = 1.0 / (np.arange(n_genes) + 1.0) ** 1.1          # power-law gene rates
    rate = rate / rate.sum()
    lib = rng.lognormal(np.log(60.0 * n_genes), 0.5, size=n_cells)
    x = rng.poisson(lib[:, None] * rate[None, :])
    return np.clip(np.maximum(x, 1), 1, 65535)


@pytest.mark.parametrize("n_genes", [512, 2000])
def test_scores_within_the_certified_bound(n_genes):
    seed = 11
    X = adversarial(4096, n_genes, seed)
    say("bound test: G", n_genes, "counts > 255:", int((X > 255).sum()), "of", X.size)
    assert (X > 255).any() and X.min() >= 1
    d = synth.from_dense(X)
    kw = dict(alpha=1.0, beta=1.0, seed=seed, k_max=16)
    s = Sampler(d.row_ptr, d.col, d.val, n_genes, k_init=1, precision="split_bf16", **kw)
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, n_genes, init=False, **kw)
    rng = np.random.default_rng(seed)
    K = 4
    c = rng.integers(0, K, size=d.n_cells).astype(np.int32)
    cs = rng.integers(0, 2, size=d.n_cells).astype(np.uint8)
    reset = np.zeros(K, dtype=np.uint8)
    s.set_state(3, K, torch.from_numpy(c), torch.from_numpy(cs), reset)
    o.set_state(3, K, c, cs, reset)
    assert o._st.flags & oracle.NEW_CLUSTER
    o.extend()
    o.redraw()
    Ks = o.K
    ref = o.cell_logliks(np.arange(d.n_cells, dtype=np.int64))[:, :Ks]
    dbg = s.debug_scores(Ks, fp64=True)
    s.sweep(1)
    s.debug_scores(None)
    got = dbg[:, :Ks].cpu().numpy()
    n = np.diff(rp).astype(np.float64)[:, None]
    bnd = (2.0 ** -17 + (2 * n + 8) * 2.0 ** -23) * 1.01 * (np.abs(got) + 20.0) + 1e-5
    err = np.abs(got - ref)
    ratio = float((err / bnd).max())
    rel = float((err / np.maximum(1.0, np.abs(ref))).max())
    say(f"bound test: G {n_genes}, K {Ks}, max |S - S64| / bound {ratio:.3e}, max relative error {rel:.3e}, "
        f"log theta down to {o.logtheta_clusters()[:Ks].min():.1f}")
    report(dict(test=f"bound-G{n_genes}", max_err_over_bound=ratio, max_rel_err=rel, cells=d.n_cells, K=Ks,
                min_log_theta=float(o.logtheta_clusters()[:Ks].min())))
    assert np.all(err <= bnd), ratio
    assert o.logtheta_clusters()[:Ks].min() < -10.0          # the prior-drawn cluster reaches far down
