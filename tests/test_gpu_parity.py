"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Both sides start from the same seeded data and the same state, draw the same
Philox numbers, and are compared step by step:
  * a1  log pi and log theta: |gpu - oracle| <= 1e-9 max(1, |oracle|)
  * a2  FP32 log-likelihoods (debug dump): |gpu - oracle| <= 1e-4 |oracle|
  * a3  labels: bit-exact except cells whose oracle Gumbel-max margin is
        below 1e-6 (counted; the GPU re-scores uncertain decisions in FP64)
  * a4  statistics: bit-exact whenever the labels are
  * a5  log R: |gpu - oracle| <= 1e-9 x (sum of the magnitudes of its terms);
        accept flags and resulting labels equal
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu

MARGIN = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sampler(d, precision, **kw):
    return Sampler(d.row_ptr, d.col, d.val, d.n_genes, precision=precision, **kw)


def _oracle(d, **kw):
    rp, col, val = d.host_arrays()
    return oracle.Oracle(rp, col, val, d.n_genes, **kw)


def _labels(s):
    c, cs = s.labels()
    return c.cpu().numpy(), cs.cpu().numpy()


def _compare_labels(o, s, what):
    c, cs = _labels(s)
    bad_c = np.nonzero(c != o.c)[0]
    bad_s = np.nonzero((c == o.c) & (cs != o.cs))[0]
    # every mismatch must be a decision the oracle itself took by less than the margin
    assert np.all(o.margin_c[bad_c] < MARGIN), (what, bad_c[:10], o.margin_c[bad_c][:10])
    assert np.all(o.margin_s[bad_s] < MARGIN), (what, bad_s[:10], o.margin_s[bad_s][:10])
    return len(bad_c) + len(bad_s)


def _compare_stats(o, s):
    st = s.stats(with_tables=True)
    K = st["K"]
    assert K == o.K
    assert np.array_equal(st["nsub"], o.nsub[: 2 * K])
    assert np.array_equal(st["ssub"].cpu().numpy(), o.ssub[: 2 * K])
    return st


def _compare_params(o, s):
    K = o.K
    lp, lt = s.params()
    lp = lp.cpu().numpy()[:K]
    lt = lt.cpu().numpy()
    ref_lp = o.logpi[:K]
    assert np.all(np.abs(lp - ref_lp) <= 1e-9 * np.maximum(1.0, np.abs(ref_lp)))
    gc = lt[:K]
    gs = lt[o.k_max: o.k_max + 2 * K]
    rc = o.logtheta[:K]
    rs = o.logtheta[o.k_max: o.k_max + 2 * K]
    err_c = np.max(np.abs(gc - rc) / np.maximum(1.0, np.abs(rc)))
    err_s = np.max(np.abs(gs - rs) / np.maximum(1.0, np.abs(rs)))
    assert err_c <= 1e-9 and err_s <= 1e-9, (err_c, err_s)
    return max(err_c, err_s)


def _compare_hastings(o, s):
    p, logr, acc = s.hastings()
    assert p == o.sm_pass
    n = o.sm_n
    assert len(logr) == n
    ref = o.sm_logr[:n]
    scale = o.sm_scale[:n]
    nan_ref = np.isnan(ref)
    assert np.array_equal(np.isnan(logr), nan_ref)
    ok = ~nan_ref
    err = np.abs(logr[ok] - ref[ok]) / np.maximum(1.0, scale[ok])
    assert np.all(err <= 1e-9), err.max()
    assert np.array_equal(acc, o.sm_accept[:n])
    return float(err.max()) if err.size else 0.0


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k_init", [1, 5])
def test_init_state_matches_oracle(k_init):
    _say("init", k_init)
    d = synth.generate("c1", seed=2, n_cells=700)
    o = _oracle(d, seed=3, k_max=32, k_init=k_init)
    s = _sampler(d, "fp32", seed=3, k_max=32, k_init=k_init)
    c, cs = _labels(s)
    assert np.array_equal(c, o.c) and np.array_equal(cs, o.cs)
    _compare_stats(o, s)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
def test_chain_lockstep_small_recipe(precision):
    """Two independent chains, one per implementation, from the same seed:
    identical at every sweep and split/merge while no near-tie occurs."""
    _say("lockstep", precision)
    d = synth.generate("c1", seed=0)
    kw = dict(alpha=1.0, beta=1.0, seed=11, k_max=64, k_init=1)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    compared = 0
    for it in range(25):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        if _compare_labels(o, s, f"sweep {it}"):
            _say("near-tie divergence at sweep", it)
            break
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        if _compare_labels(o, s, f"split/merge {it}"):
            break
        _compare_stats(o, s)
        compared += 1
    assert compared >= 10
    st = s.stats()
    _say("K", st["K"], "refined", st["refined"], "splits", st["splits_accepted"], "merges", st["merges_accepted"])


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_split_q_chain_lockstep(precision):
    """With the split proposal term (DPMM_FLAG_SPLIT_Q, Section 2.3) on both
    sides: split ratios within the condition-aware tolerance of the oracle's,
    the same accept decisions and labels, for several split passes."""
    _say("split_q lockstep", precision)
    d = synth.generate("c1", seed=4)
    kw = dict(alpha=1.0, beta=1.0, seed=17, k_max=64, k_init=1)
    o = _oracle(d, split_q=True, **kw)
    s = _sampler(d, precision, split_q=True, **kw)
    splits = 0
    for it in range(25):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        if _compare_labels(o, s, f"sweep {it}"):
            break
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        if o.sm_pass == 0 and np.any(~np.isnan(o.sm_logr[: o.sm_n])):
            splits += 1
        if _compare_labels(o, s, f"split/merge {it}"):
            break
        _compare_stats(o, s)
    assert splits >= 2
    _say("K", s.stats()["K"], "split passes compared", splits)


def _three_groups():
    rng = np.random.default_rng(13)
    grp = np.repeat(np.arange(3), 40)
    X = rng.poisson(0.3, size=(120, 3))
    X[np.arange(120), grp] += 8
    return synth.from_dense(X)


@pytest.mark.parametrize("case", ["three_groups-fp64", "three_groups-split_bf16", "c1-fp32"])
def test_new_cluster_chain_lockstep(case):
    """With the Gibbs step over K + 1 clusters (DPMM_FLAG_NEW_CLUSTER, eq. 4) on
    both sides (and the split proposal term on c1): parameters, labels,
    statistics and Hastings ratios in lockstep with the oracle; on the
    three-group data the Gibbs step itself opens clusters."""
    data, precision = case.split("-")
    _say("new_cluster lockstep", case)
    if data == "c1":
        d = synth.generate("c1", seed=7)
        kw = dict(alpha=1.0, beta=1.0, seed=23, k_max=64, k_init=1, new_cluster=True, split_q=True)
    else:
        d = _three_groups()
        kw = dict(alpha=2.0, beta=0.2, seed=9, k_max=16, k_init=1, new_cluster=True)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    opened = 0
    compared = 0
    for it in range(30):
        k0 = o.K
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        if _compare_labels(o, s, f"sweep {it}"):
            break
        _compare_stats(o, s)
        opened += o.K > k0
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        if _compare_labels(o, s, f"split/merge {it}"):
            break
        _compare_stats(o, s)
        compared += 1
    assert compared >= 10
    if data == "three_groups":
        assert opened >= 1
    _say("K", s.stats()["K"], "sweeps that opened a cluster", opened)


@pytest.mark.parametrize("case", ["c1-split_bf16", "c1-fp64", "tiny-fp64"])
def test_random_split_chain_lockstep(case):
    """With the random-split pass (DPMM_FLAG_RANDOM_SPLIT, chain B of Section
    2.4) on both sides: the pass chosen, the ratios of every pass, the accept
    decisions, labels and statistics in lockstep with the oracle; on the tiny
    high-alpha data random splits are accepted."""
    data, precision = case.split("-")
    _say("random_split lockstep", case)
    if data == "c1":
        d = synth.generate("c1", seed=12)
        kw = dict(alpha=1.0, beta=1.0, seed=31, k_max=64, k_init=1, random_split=True)
    else:
        X = np.random.default_rng(3).integers(1, 4, size=(24, 3))
        d = synth.from_dense(X)
        kw = dict(alpha=200.0, beta=1.0, seed=5, k_max=16, k_init=1, random_split=True)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    rpasses = accepted = 0
    for it in range(30):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        if _compare_labels(o, s, f"sweep {it}"):
            break
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        if o.sm_pass == 2:
            rpasses += 1
            accepted += int(o.sm_accept[: o.sm_n].sum())
        if _compare_labels(o, s, f"split/merge {it}"):
            break
        _compare_stats(o, s)
    assert rpasses >= 3
    if data == "tiny":
        assert accepted >= 1
    _say("K", s.stats()["K"], "random passes", rpasses, "accepted", accepted)


SCORE_TOL = {"fp32": 1e-4, "split_bf16": 3e-5}


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_sweep_at_68k_cells_matches_oracle(precision):
    """The 68,000 x 1,000 recipe: one sweep and one split/merge from a state
    reached by the oracle, with the log-likelihoods checked cell by cell
    (FP32: 1e-4 relative; split-BF16: 3e-5 relative, its certified bound is
    about 1.5e-5)."""
    _say("c2 full size", precision)
    d = synth.generate("c2", seed=0)
    kw = dict(alpha=1.0, beta=1.0, seed=5, k_max=64)
    o = _oracle(d, k_init=1, **kw)
    o.iterate(6)
    snap = o.snapshot()
    s = _sampler(d, precision, k_init=1, **kw)
    s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    _compare_stats(o, s)
    K = o.K
    dbg = s.debug_scores(K)
    o.sweep()
    s.sweep(1)
    _compare_params(o, s)
    mism = _compare_labels(o, s, "c2 sweep")
    if mism == 0:
        _compare_stats(o, s)
    # FP32 log-likelihoods of a sample of cells against FP64
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(d.n_cells, size=3000, replace=False))
    ref = o.cell_logliks(cells)
    got = dbg.cpu().numpy()[cells]
    K2 = o.K
    assert K2 <= K
    gk = got[:, :K2]
    rk = ref[:, :K2]
    tol = SCORE_TOL[precision]
    rel = np.abs(gk - rk) / np.maximum(1.0, np.abs(rk))
    _say("max relative log-likelihood error", float(rel.max()), "median", float(np.median(rel)))
    assert np.all(np.abs(gk - rk) <= tol * np.abs(rk) + 1e-3)
    live = ~np.isnan(got[:, K2])   # cells of clusters not flagged for reset
    # the two sub-cluster scores are FP64 in every precision
    assert np.all(np.abs(got[live, K2:K2 + 2] - ref[live, K2:K2 + 2]) <= 1e-6 * np.abs(ref[live, K2:K2 + 2]) + 1e-3)
    s.debug_scores(None)
    o.split_merge()
    s.split_merge()
    if mism == 0:
        _compare_hastings(o, s)
        _compare_labels(o, s, "c2 split/merge")
        _compare_stats(o, s)
    _say("c2 mismatches", mism, "refined", s.stats()["refined"])


def test_empirical_bayes_step_matches_oracle():
    _say("eb")
    d = synth.generate("c1", seed=4, n_cells=1200)
    kw = dict(alpha=1.0, beta=0.5, seed=9, k_max=32)
    o = _oracle(d, k_init=1, **kw)
    o.iterate(8)
    snap = o.snapshot()
    s = _sampler(d, "fp32", k_init=1, **kw)
    s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    for _ in range(3):
        o.eb_update()
        s.eb_update()
        b = s.beta.cpu().numpy()
        assert np.all(np.abs(b - o.beta) <= 1e-9 * np.abs(o.beta)), np.max(np.abs(b - o.beta) / o.beta)
    # the Hastings sums read per-gene log-gamma tables, which must follow beta
    # wherever it is written: after the EB steps, and after set_beta
    o.split_merge()
    s.split_merge()
    _compare_hastings(o, s)
    assert _compare_labels(o, s, "eb split/merge") == 0
    nb = np.random.default_rng(3).uniform(0.05, 3.0, size=d.n_genes)
    o.beta[:] = nb
    s.beta = torch.from_numpy(nb).cuda()
    for it in range(2):
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        assert _compare_labels(o, s, f"set_beta split/merge {it}") == 0


def test_dm_logmarginal_and_gradient_match_oracle():
    _say("dm")
    from paper_1812_10048_amd.sampler import DMLogMarginal
    rng = np.random.default_rng(1)
    J, G = 36, 2000
    s_np = rng.negative_binomial(0.3, 0.01, size=(J, G)).astype(np.int64)
    s_np[rng.random((J, G)) < 0.5] = 0
    beta_np = rng.uniform(0.05, 3.0, size=G)
    g_np = rng.normal(size=J)
    beta = torch.tensor(beta_np, device="cuda", requires_grad=True)
    s_t = torch.tensor(s_np, device="cuda")
    out = DMLogMarginal.apply(beta, s_t)
    ref = oracle.dm_logmarginal(s_np, beta_np)
    assert np.all(np.abs(out.detach().cpu().numpy() - ref) <= 1e-9 * np.abs(ref))
    (out * torch.tensor(g_np, device="cuda")).sum().backward()
    gref = oracle.dm_grad(s_np, beta_np, g_np)
    got = beta.grad.cpu().numpy()
    assert np.all(np.abs(got - gref) <= 1e-9 * np.maximum(1.0, np.abs(gref)))


def test_edge_cases():
    _say("edges")
    # a cell with no counts, a single gene, a single cell
    X = np.array([[0, 3, 1], [0, 0, 0], [5, 0, 2], [1, 1, 1]])
    d = synth.from_dense(X)
    for prec in ("fp64", "fp32", "split_bf16"):
        o = _oracle(d, seed=1, k_max=4, k_init=2)
        s = _sampler(d, prec, seed=1, k_max=4, k_init=2)
        for _ in range(6):
            o.sweep(); s.sweep(1)
            assert _compare_labels(o, s, "edge") == 0
            _compare_stats(o, s)
            o.split_merge(); s.split_merge()
            assert _compare_labels(o, s, "edge sm") == 0
    d1 = synth.from_dense(np.array([[7]]))
    s = _sampler(d1, "fp32", seed=0, k_max=2)
    s.iterate(3)
    assert s.K == 1
    # invalid CSR content is reported, not crashed on
    from paper_1812_10048_amd import dpmm as C
    bad_col = torch.tensor([0, 5], dtype=torch.int32)
    with pytest.raises(C.DpmmError) as e:
        Sampler(torch.tensor([0, 2]), bad_col, torch.tensor([1, 1], dtype=torch.int32), 3)
    assert e.value.status == C.DPMM_ERR_DATA
    with pytest.raises(C.DpmmError) as e:
        Sampler(torch.tensor([0, 2]), torch.tensor([1, 1], dtype=torch.int32), torch.tensor([1, 1], dtype=torch.int32), 3)
    assert e.value.status == C.DPMM_ERR_DATA


def test_capacity_limit_counts_skipped_splits():
    _say("kmax")
    d = synth.generate("c1", seed=0, n_cells=600)
    kw = dict(alpha=1.0, beta=1.0, seed=11, k_max=2, k_init=1)
    o = _oracle(d, **kw)
    s = _sampler(d, "fp32", **kw)
    for _ in range(12):
        o.iterate(1)
        s.iterate(1)
        assert _compare_labels(o, s, "kmax") == 0
    assert s.K <= 2
    assert s.stats()["kmax_skips"] == o.counters()["kmax_skips"]


def test_resume_reproduces_the_chain():
    _say("resume")
    d = synth.generate("c1", seed=1, n_cells=900)
    kw = dict(alpha=1.0, beta=0.7, seed=21, k_max=32, k_init=3)
    a = _sampler(d, "fp32", **kw)
    a.iterate(8, eb_every=3)
    b = _sampler(d, "fp32", **kw)
    b.iterate(4, eb_every=3)
    snap = b.snapshot()
    r = _sampler(d, "fp32", **kw)
    r.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    r.beta = snap["beta"]
    # continue both with the same schedule as the uninterrupted chain
    for it in range(4, 8):
        for x in (b, r):
            x.iterate(1)
            if (it + 1) % 3 == 0:
                x.eb_update()
    for x in (b, r):
        cx, csx = _labels(x)
        ca, csa = _labels(a)
        assert np.array_equal(cx, ca) and np.array_equal(csx, csa)


@pytest.mark.parametrize("precision", ["fp32", "fp64", "split_bf16"])
@pytest.mark.parametrize("k_init", [12, 24, 40, 56, 70])
def test_many_cluster_kernel_paths(precision, k_init):
    """Cluster counts that select each register-tile width of the assignment
    kernel, its cluster-group loop (K > 64) and the gathered sub-cluster pass."""
    _say("paths", precision, k_init)
    d = synth.generate("c1", seed=6, n_cells=3000)
    kw = dict(alpha=1.0, beta=1.0, seed=13, k_max=96, k_init=k_init)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    assert o.K == s.K == k_init
    for it in range(2):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        assert _compare_labels(o, s, f"paths sweep {it}") == 0
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        assert _compare_labels(o, s, f"paths sm {it}") == 0
        _compare_stats(o, s)


def test_split_bf16_tables_are_hi_lo_of_log_theta():
    """Row a8: hi = bf16(fp32(log theta)), lo = bf16(fp32(log theta - hi)),
    round to nearest even, and |log theta - hi - lo| <= 2^-17 |log theta|."""
    _say("split tables")
    d = synth.generate("c1", seed=3, n_cells=1500)
    s = _sampler(d, "split_bf16", seed=4, k_max=16, k_init=3, beta=0.3)
    s.sweep(2)
    K = s.K
    _, lt = s.params()
    lt = lt[:K]
    hi, lo = s.split_tables()
    hi_f = hi.view(torch.bfloat16).float().double()
    lo_f = lo.view(torch.bfloat16).float().double()
    exp_hi = lt.float().bfloat16()
    assert torch.equal(hi.view(torch.bfloat16), exp_hi)
    exp_lo = (lt - exp_hi.double()).float().bfloat16()
    assert torch.equal(lo.view(torch.bfloat16), exp_lo)
    resid = (lt - hi_f - lo_f).abs()
    assert bool((resid <= 2.0 ** -17 * lt.abs() + 1e-300).all())


@pytest.mark.parametrize("n_genes", [6000, 20000])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
def test_wide_matrices_take_the_global_memory_paths(precision, n_genes):
    """More genes than the LDS tables hold: above 4096 the sub-cluster pass
    reads its parameters from global memory, above 8192 its histograms are
    global atomics, above 16384 the initial statistics use the atomic kernel;
    the split-BF16 kernel walks a few hundred gene chunks."""
    _say("wide", precision, n_genes)
    rec = synth.Recipe("wide", 2500, n_genes, "fixed:900,700,500,400", 0.02, 3000.0, 0.5)
    d = synth.generate(rec, seed=3)
    kw = dict(alpha=1.0, beta=1.0, seed=17, k_max=16, k_init=3)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    _compare_stats(o, s)
    for it in range(3):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        if _compare_labels(o, s, f"wide sweep {it}"):
            break
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        if _compare_labels(o, s, f"wide sm {it}"):
            break
        _compare_stats(o, s)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_two_hundred_clusters(precision):
    """About 200 clusters of k_max = 256, started from the true partition of
    a 200-cluster matrix: several column groups in both assignment kernels and
    ~20k merge candidates in the single-workgroup decision."""
    _say("k200", precision)
    rec = synth.Recipe("k200", 20000, 500, "dirichlet:200", 0.05, 2000.0, 0.5)
    d = synth.generate(rec, seed=8)
    kw = dict(alpha=1.0, beta=1.0, seed=19, k_max=256, k_init=1)
    o = _oracle(d, **kw)
    s = _sampler(d, precision, **kw)
    cs0 = np.random.default_rng(2).integers(0, 2, size=d.n_cells)
    reset = np.ones(d.n_true, dtype=np.uint8)
    o.set_state(0, d.n_true, d.z, cs0, reset)
    s.set_state(0, d.n_true, torch.from_numpy(d.z), torch.from_numpy(cs0), reset)
    _compare_stats(o, s)
    assert o.K > 150
    merges = 0
    for it in range(4):
        o.sweep()
        s.sweep(1)
        _compare_params(o, s)
        assert _compare_labels(o, s, f"k200 sweep {it}") == 0
        _compare_stats(o, s)
        o.split_merge()
        s.split_merge()
        _compare_hastings(o, s)
        merges += o.sm_pass == 1
        assert _compare_labels(o, s, f"k200 sm {it}") == 0
        _compare_stats(o, s)
    _say("k200 K", o.K, "merge passes", merges)
