"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Both sides start from the same seeded data and the same state, draw the same
Philox numbers, and are compared step by step by ``lockstep.Lockstep``:
  * a1  log pi and log theta: |gpu - oracle| <= 1e-9 max(1, |oracle|)
  * a2  log-likelihoods: the sweep's own FP64 scores within 1e-9, FP32 within
        1e-4 relative, split-BF16 within 3e-5 relative, every cell of the
        68k-cell recipe; FP64 listed-cell dumps within 1e-9
  * a3  labels: bit-exact except cells whose oracle Gumbel-max margin is
        below 1e-6 (the chains are then re-synchronised and go on); the
        near-tie counter equal to the oracle's count
  * a4  statistics: bit-exact after every step; the log joint within 1e-9
  * a5  log R: |gpu - oracle| <= 1e-9 x (sum of the magnitudes of its terms);
        accept flags and resulting labels equal
"""
import numpy as np
import pytest
import torch

import oracle
from lockstep import Lockstep, say
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu

# the plain passes (one fair coin: sub-cluster split or merge), flags = 0
COLLAPSED = dict(split_q=False, new_cluster=False, random_split=False)


def _sampler(d, precision, **kw):
    return Sampler(d.row_ptr, d.col, d.val, d.n_genes, precision=precision, **kw)


def _oracle(d, **kw):
    rp, col, val = d.host_arrays()
    return oracle.Oracle(rp, col, val, d.n_genes, **kw)


def _pair(d, precision, **kw):
    return _oracle(d, **kw), _sampler(d, precision, **kw)


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k_init", [1, 5])
def test_init_state_matches_oracle(k_init):
    say("init", k_init)
    d = synth.generate("c1", seed=2, n_cells=700)
    o, s = _pair(d, "fp32", seed=3, k_max=32, k_init=k_init)
    c, cs = s.labels()
    assert np.array_equal(c.cpu().numpy(), o.c) and np.array_equal(cs.cpu().numpy(), o.cs)
    Lockstep("init", o, s).compare_stats()


@pytest.mark.parametrize("moves", ["paper", "collapsed"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
def test_chain_lockstep_small_recipe(precision, moves):
    """Two chains, one per implementation, from the same seed: compared at
    every sweep and split/merge for 25 iterations from one cluster."""
    say("lockstep", precision, moves)
    d = synth.generate("c1", seed=0)
    kw = dict(alpha=1.0, beta=1.0, seed=11, k_max=64, k_init=1, **(COLLAPSED if moves == "collapsed" else {}))
    ls = Lockstep(f"c1-{precision}-{moves}", *_pair(d, precision, **kw))
    ls.iterate(25)
    ls.finish()
    assert ls.o.K >= 3


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_split_q_chain_lockstep(precision):
    """The split proposal term alone (DPMM_FLAG_SPLIT_Q, Section 2.3): split
    ratios, decisions and labels in lockstep, several split passes."""
    say("split_q lockstep", precision)
    d = synth.generate("c1", seed=4)
    kw = dict(alpha=1.0, beta=1.0, seed=17, k_max=64, k_init=1, **{**COLLAPSED, "split_q": True})
    ls = Lockstep(f"split_q-{precision}", *_pair(d, precision, **kw))
    ls.iterate(25)
    ls.finish()
    assert ls.passes[0] >= 2


def _three_groups():
    rng = np.random.default_rng(13)
    grp = np.repeat(np.arange(3), 40)
    X = rng.poisson(0.3, size=(120, 3))
    X[np.arange(120), grp] += 8
    return synth.from_dense(X)


@pytest.mark.parametrize("case", ["three_groups-fp64", "three_groups-split_bf16", "c1-fp32"])
def test_new_cluster_chain_lockstep(case):
    """The Gibbs step over K + 1 clusters (DPMM_FLAG_NEW_CLUSTER, eq. 4) on both
    sides (with the split proposal term on c1); on the three-group data the
    Gibbs step itself opens clusters."""
    data, precision = case.split("-")
    say("new_cluster lockstep", case)
    if data == "c1":
        d = synth.generate("c1", seed=7)
        kw = dict(alpha=1.0, beta=1.0, seed=23, k_max=64, k_init=1,
                  **{**COLLAPSED, "new_cluster": True, "split_q": True})
    else:
        d = _three_groups()
        kw = dict(alpha=2.0, beta=0.2, seed=9, k_max=16, k_init=1, **{**COLLAPSED, "new_cluster": True})
    ls = Lockstep(f"new_cluster-{case}", *_pair(d, precision, **kw))
    opened = 0
    for it in range(30):
        k0 = ls.o.K
        ls.sweep()
        opened += ls.o.K > k0
        ls.split_merge()
    ls.finish(opened=opened)
    if data == "three_groups":
        assert opened >= 1


@pytest.mark.parametrize("case", ["c1-split_bf16", "c1-fp64", "tiny-fp64", "tiny-fp64-twice"])
def test_random_split_chain_lockstep(case):
    """The random-split pass (DPMM_FLAG_RANDOM_SPLIT, chain B of Section 2.4):
    the pass chosen, every ratio, the decisions, labels and statistics; on the
    tiny high-alpha data random splits are accepted.  A random split right
    after a sweep takes its coins and coin halves from the sweep's sub-cluster
    pass; "twice" makes two split/merge calls per sweep, so that the second
    one builds them with a pass of its own."""
    data, precision, *mode = case.split("-")
    calls = 2 if mode == ["twice"] else 1
    say("random_split lockstep", case)
    if data == "c1":
        d = synth.generate("c1", seed=12)
        kw = dict(alpha=1.0, beta=1.0, seed=31, k_max=64, k_init=1, **{**COLLAPSED, "random_split": True})
    else:
        X = np.random.default_rng(3).integers(1, 4, size=(24, 3))
        d = synth.from_dense(X)
        kw = dict(alpha=200.0, beta=1.0, seed=5, k_max=16, k_init=1, **{**COLLAPSED, "random_split": True})
    ls = Lockstep(f"random_split-{case}", *_pair(d, precision, **kw))
    accepted_random = 0
    for it in range(30):
        ls.sweep()
        for _ in range(calls):
            ls.split_merge()
            if ls.o.sm_pass == 2:
                accepted_random += int(ls.o.sm_accept[: ls.o.sm_n].sum())
    ls.finish(accepted_random=accepted_random)
    assert ls.passes[2] >= 3
    if data == "tiny":
        assert accepted_random >= 1


SCORE_TOL = {"fp32": 1e-4, "split_bf16": 3e-5}


def _sweep_columns(o, K):
    """Clusters of a sweep that started with K: K + 1 when the Gibbs step runs
    over a new cluster (eq. 4) and there is room for it, else K."""
    return K + 1 if (o._st.flags & oracle.NEW_CLUSTER) and K < o.k_max else K


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_sweep_at_68k_cells_matches_oracle(precision):
    """The 68,000 x 1,000 recipe at full size: two sweeps and split/merge calls
    from a state the oracle reached, with the sweep's own log-likelihoods of
    every cell checked against FP64 (FP32 1e-4 relative, split-BF16 3e-5
    relative; the sub-cluster scores are FP64 in both and checked at 1e-9 in
    the second sweep, when no cluster re-draws its sub-labels), and the FP64
    listed-cell dump at 1e-9."""
    say("c2 full size", precision)
    d = synth.generate("c2", seed=0)
    kw = dict(alpha=1.0, beta=1.0, seed=5, k_max=64)
    o = _oracle(d, k_init=1, **kw)
    o.iterate(6)
    snap = o.snapshot()
    s = _sampler(d, precision, k_init=1, **kw)
    s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    o.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    ls = Lockstep(f"c2-{precision}", o, s)
    ls.compare_stats()
    worst = {}
    for sweep in range(2):
        K = o.K
        dbg = s.debug_scores(K + 1, fp64=True)       # room for the new cluster of eq. 4
        ls.sweep()
        s.debug_scores(None)
        got = dbg.cpu().numpy()
        Ks, K2 = _sweep_columns(o, K), o.K
        ref = o.cell_logliks(np.arange(d.n_cells))
        Kc = min(Ks, K2)
        gk, rk = got[:, :Kc], ref[:, :Kc]
        rel = np.abs(gk - rk) / np.maximum(1.0, np.abs(rk))
        worst[f"cluster_rel_err_sweep{sweep}"] = float(rel.max())
        assert np.all(np.abs(gk - rk) <= SCORE_TOL[precision] * np.abs(rk) + 1e-3)
        live = ~np.isnan(got[:, Ks])
        if sweep == 1:
            assert live.mean() > 0.99          # no cluster re-drew its sub-labels
        if K2 >= K:                            # no cluster of the sweep renumbered
            sub_err = (np.abs(got[live, Ks:Ks + 2] - ref[live, K2:K2 + 2]) /
                       np.maximum(1.0, np.abs(ref[live, K2:K2 + 2])))
            worst[f"sub_rel_err_sweep{sweep}"] = float(sub_err.max(initial=0.0))
            assert np.all(sub_err <= 1e-9)
        # FP64 dump of listed cells: one per block of 256 and the last cell
        pick = np.unique(np.r_[np.arange(0, d.n_cells, 256), d.n_cells - 1]).astype(np.int32)
        dump = s.dump_scores(pick).cpu().numpy()
        dref = ref[pick]
        assert np.all(np.abs(dump - dref) <= 1e-9 * np.maximum(1.0, np.abs(dref)))
        ls.split_merge()
    ls.finish(**worst)


def test_fp64_sweep_scores_match_at_fp64_tolerance():
    """The FP64 precision: the sweep's own cluster and sub-cluster scores of
    every cell within 1e-9 relative of the oracle's."""
    say("fp64 scores")
    d = synth.generate("c1", seed=5)
    kw = dict(alpha=1.0, beta=1.0, seed=3, k_max=32, k_init=4)
    o, s = _pair(d, "fp64", **kw)
    ls = Lockstep("fp64-scores", o, s)
    checked = 0
    for sweep in range(4):
        K = o.K
        dbg = s.debug_scores(K + 1, fp64=True)
        ls.sweep()
        s.debug_scores(None)
        got = dbg.cpu().numpy()
        Ks, K2 = _sweep_columns(o, K), o.K
        ref = o.cell_logliks(np.arange(d.n_cells))
        Kc = min(Ks, K2)
        assert np.all(np.abs(got[:, :Kc] - ref[:, :Kc]) <= 1e-9 * np.maximum(1.0, np.abs(ref[:, :Kc])))
        if K2 >= K:
            live = ~np.isnan(got[:, Ks])
            g, r = got[live, Ks:Ks + 2], ref[live, K2:K2 + 2]
            assert np.all(np.abs(g - r) <= 1e-9 * np.maximum(1.0, np.abs(r)))
            checked += int(live.sum())
        ls.split_merge()
    ls.finish(sub_scores_checked=checked)
    assert checked > 0


def test_empirical_bayes_step_matches_oracle():
    say("eb")
    d = synth.generate("c1", seed=4, n_cells=1200)
    kw = dict(alpha=1.0, beta=0.5, seed=9, k_max=32)
    o = _oracle(d, k_init=1, **kw)
    o.iterate(8)
    snap = o.snapshot()
    s = _sampler(d, "fp32", k_init=1, **kw)
    s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    o.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    ls = Lockstep("eb", o, s)
    for _ in range(3):
        o.eb_update()
        s.eb_update()
        b = s.beta.cpu().numpy()
        assert np.all(np.abs(b - o.beta) <= 1e-9 * np.abs(o.beta)), np.max(np.abs(b - o.beta) / o.beta)
    # the Hastings sums read per-gene log-gamma tables, which must follow beta
    # wherever it is written: after the EB steps, and after set_beta
    ls.split_merge()
    nb = np.random.default_rng(3).uniform(0.05, 3.0, size=d.n_genes)
    o.beta[:] = nb
    s.beta = torch.from_numpy(nb).cuda()
    for it in range(2):
        ls.split_merge()
    ls.finish()


def test_dm_logmarginal_and_gradient_match_oracle():
    say("dm")
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
    say("edges")
    # a cell with no counts, a single gene, a single cell
    X = np.array([[0, 3, 1], [0, 0, 0], [5, 0, 2], [1, 1, 1]])
    d = synth.from_dense(X)
    for prec in ("fp64", "fp32", "split_bf16"):
        ls = Lockstep(f"edge-{prec}", *_pair(d, prec, seed=1, k_max=4, k_init=2))
        ls.iterate(6)
        ls.finish()
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
    # the FP64 dump needs parameters drawn by a sweep
    s2 = _sampler(d, "fp32", seed=1, k_max=4, k_init=2)
    with pytest.raises(C.DpmmError) as e:
        s2.dump_scores([0, 1])
    assert e.value.status == C.DPMM_ERR_STATE


def _big_counts(seed: int = 5) -> np.ndarray:
    """Three groups of cells (ragged blocks of 256), each dense on its own 90
    genes, with about 30 % of those counts at or above 256 (up to the largest
    count a packed entry holds, 65,535) and some at exactly 255; a cell with no
    counts and a cell whose one count is 65,535.  In any partition, a block's
    cluster then has counts above 255 on its first 32 places (split into a low
    byte and a high plane), on places 32-63 (tail entries beside the dense
    chunk) and on genes past the dense chunks."""
    rng = np.random.default_rng(seed)
    sizes, G, width = (260, 300, 180), 300, 90
    big = np.array([255, 256, 257, 300, 511, 512, 1000, 4095, 65535])
    rows = []
    for g, n in enumerate(sizes):
        x = rng.poisson(0.2, size=(n, G))
        x[:, g * width:(g + 1) * width] = rng.poisson(20.0, size=(n, width)) + 1
        hit = rng.random((n, width)) < 0.3
        blk = x[:, g * width:(g + 1) * width]
        blk[hit] = rng.choice(big, size=int(hit.sum()))
        rows.append(x)
    x = np.concatenate(rows)
    x[5] = 0
    x[7] = 0
    x[7, 3] = 65535
    return x


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_bf16"])
def test_counts_above_255_on_the_top_genes(precision):
    """Large counts where the split-BF16 copy splits them (the high plane),
    keeps them in the tail beside a dense chunk, or past the dense chunks:
    labels, statistics and split/merge decisions in lockstep with the
    oracle (eq. 26 for the scores, eq. 8 and the sufficient statistics)."""
    say(f"bigcounts-{precision}")
    d = synth.from_dense(_big_counts())
    ls = Lockstep(f"bigcounts-{precision}", *_pair(d, precision, seed=3, k_max=16, k_init=2))
    ls.iterate(8)
    ls.finish()


def test_capacity_limit_counts_skipped_splits():
    say("kmax")
    d = synth.generate("c1", seed=0, n_cells=600)
    kw = dict(alpha=1.0, beta=1.0, seed=11, k_max=2, k_init=1)
    ls = Lockstep("kmax", *_pair(d, "fp32", **kw))
    ls.iterate(12)
    ls.finish()
    assert ls.s.K <= 2
    assert ls.s.stats()["kmax_skips"] == ls.o.counters()["kmax_skips"]


def test_resume_reproduces_the_chain():
    """A chain resumed from (step, K, c, cbar, reset, beta) saved between two
    iterations continues exactly as the uninterrupted one (every cell's eq. 8
    probability is redrawn by the sweep before the next split pass reads it)."""
    say("resume")
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
    ca, csa = a.labels()
    for x in (b, r):
        cx, csx = x.labels()
        assert torch.equal(cx, ca) and torch.equal(csx, csa)


@pytest.mark.parametrize("precision", ["split_bf16", "fp32", "fp64"])
def test_two_runs_agree_bit_for_bit(precision):
    """Run-to-run determinism: the same chain twice from the same seed gives the
    same labels, statistics, log pi and log theta bit for bit, and the same
    per-cell scores in the debug dump of a sweep; log R (FP64 sums, some
    gathered with atomics in the split proposal term) agrees within 1e-12 of
    its magnitude, with the same pass and decisions."""
    say("determinism", precision)
    d = synth.generate("c1", seed=8)
    kw = dict(alpha=1.0, beta=1.0, seed=19, k_max=64, k_init=1)
    out = []
    for rep in range(2):
        s = _sampler(d, precision, **kw)
        s.iterate(6, eb_every=4)
        dbg = s.debug_scores(s.K + 1)
        s.sweep(1)
        s.debug_scores(None)
        s.split_merge()
        st = s.stats(with_tables=True)
        K = st["K"]
        lp, lt = s.params()
        c, cs = s.labels()
        p, logr, acc = s.hastings()
        km = kw["k_max"]
        out.append(dict(K=K, nsub=st["nsub"], ssub=st["ssub"].cpu(), lp=lp[:K].cpu(),
                        lt=torch.cat([lt[:K], lt[km:km + 2 * K]]).cpu(), c=c.cpu(), cs=cs.cpu(),
                        dbg=dbg.cpu().view(torch.int32), p=p, logr=logr, acc=acc))
        del s
    a, b = out
    assert a["K"] == b["K"] and a["K"] >= 2
    assert np.array_equal(a["nsub"], b["nsub"]) and torch.equal(a["ssub"], b["ssub"])
    assert torch.equal(a["c"], b["c"]) and torch.equal(a["cs"], b["cs"])
    assert torch.equal(a["lp"].view(torch.int64), b["lp"].view(torch.int64))
    assert torch.equal(a["lt"].view(torch.int64), b["lt"].view(torch.int64))
    assert torch.equal(a["dbg"], b["dbg"])
    assert a["p"] == b["p"] and np.array_equal(a["acc"], b["acc"])
    fa, fb = np.isfinite(a["logr"]), np.isfinite(b["logr"])
    assert np.array_equal(fa, fb)
    assert np.all(np.abs(a["logr"][fa] - b["logr"][fa]) <= 1e-12 * np.maximum(1.0, np.abs(a["logr"][fa])))


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_chain_does_not_depend_on_host_timing(precision):
    """Launch sizes follow the K the host last saw (a mapped word the device
    updates), which lags behind K when the host queues steps ahead of the GPU:
    a chain queued in one go (from one cluster, so that splits raise K while
    later steps are already queued) must equal the same chain run with a
    synchronisation after every call."""
    say("host timing", precision)
    d = synth.generate("c1", seed=2)
    kw = dict(alpha=1.0, beta=1.0, seed=41, k_max=64, k_init=1)
    a = _sampler(d, precision, **kw)
    torch.cuda.synchronize()
    # keep the stream busy (about 0.1 s of products) while the whole chain is
    # queued, so that every launch of it sees the K of the start
    m = torch.randn(8192, 8192, device="cuda")
    sink = torch.empty_like(m)
    for _ in range(10):
        torch.mm(m, m, out=sink)
    a.iterate(20, eb_every=7)
    b = _sampler(d, precision, **kw)
    for it in range(20):
        b.sweep(1)
        torch.cuda.synchronize()
        b.stats()
        b.split_merge()
        torch.cuda.synchronize()
        b.stats()
        if (it + 1) % 7 == 0:
            b.eb_update()
    sa, sb = a.stats(with_tables=True), b.stats(with_tables=True)
    assert sa["K"] == sb["K"] and sa["K"] >= 3
    assert np.array_equal(sa["nsub"], sb["nsub"])
    ca, csa = a.labels()
    cb, csb = b.labels()
    assert torch.equal(ca, cb) and torch.equal(csa, csb)
    K, km = sa["K"], kw["k_max"]
    _, lta = a.params()
    _, ltb = b.params()
    assert torch.equal(lta[:K], ltb[:K]) and torch.equal(lta[km:km + 2 * K], ltb[km:km + 2 * K])


@pytest.mark.parametrize("precision", ["fp32", "fp64", "split_bf16"])
@pytest.mark.parametrize("k_init", [12, 24, 40, 56, 70])
def test_many_cluster_kernel_paths(precision, k_init):
    """Cluster counts that select each register-tile width of the assignment
    kernel, its cluster-group loop (K > 64) and the gathered sub-cluster pass."""
    say("paths", precision, k_init)
    d = synth.generate("c1", seed=6, n_cells=3000)
    kw = dict(alpha=1.0, beta=1.0, seed=13, k_max=96, k_init=k_init)
    o, s = _pair(d, precision, **kw)
    assert o.K == s.K == k_init
    ls = Lockstep(f"paths-{precision}-{k_init}", o, s)
    ls.iterate(2)
    ls.finish()


def test_every_decision_rescored_in_the_fused_pass():
    """With refine_tol 1 every cluster decision of the split-BF16 sweep is
    uncertain, so the queue kernel of the fused sub-cluster pass re-scores each
    cell in FP64 (eq. 4) before its sub-cluster draw (eq. 8): the chain still
    matches the oracle in lockstep, and every decision is counted."""
    say("rescore all")
    d = synth.generate("c1", seed=6, n_cells=3000)
    kw = dict(alpha=1.0, beta=1.0, seed=21, k_max=32, k_init=6)
    o = _oracle(d, **kw)
    s = _sampler(d, "split_bf16", refine_tol=1.0, **kw)
    r0 = s.stats()["refined"]
    ls = Lockstep("rescore-all", o, s)
    for _ in range(3):
        K = s.K
        r1 = s.stats()["refined"]
        ls.sweep()
        if K >= 2:
            assert s.stats()["refined"] - r1 == d.n_cells
        ls.split_merge()
    ls.finish()
    assert s.stats()["refined"] > r0


def test_split_bf16_tables_are_hi_lo_of_log_theta():
    """Row a8: hi = bf16(fp32(log theta)), lo = bf16(fp32(log theta - hi)),
    round to nearest even, and |log theta - hi - lo| <= 2^-17 |log theta|."""
    say("split tables")
    d = synth.generate("c1", seed=3, n_cells=1500)
    s = _sampler(d, "split_bf16", seed=4, k_max=16, k_init=3, beta=0.3, **COLLAPSED)
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
    say("wide", precision, n_genes)
    rec = synth.Recipe("wide", 2500, n_genes, "fixed:900,700,500,400", 0.02, 3000.0, 0.5)
    d = synth.generate(rec, seed=3)
    kw = dict(alpha=1.0, beta=1.0, seed=17, k_max=16, k_init=3)
    ls = Lockstep(f"wide-{precision}-{n_genes}", *_pair(d, precision, **kw))
    ls.compare_stats()
    ls.iterate(3)
    ls.finish()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_two_hundred_clusters(precision):
    """About 200 clusters of k_max = 256, started from the true partition of
    a 200-cluster matrix: several column groups in both assignment kernels and
    ~20k merge candidates in the single-workgroup decision."""
    say("k200", precision)
    rec = synth.Recipe("k200", 20000, 500, "dirichlet:200", 0.05, 2000.0, 0.5)
    d = synth.generate(rec, seed=8)
    kw = dict(alpha=1.0, beta=1.0, seed=19, k_max=256, k_init=1)
    o, s = _pair(d, precision, **kw)
    cs0 = np.random.default_rng(2).integers(0, 2, size=d.n_cells)
    reset = np.ones(d.n_true, dtype=np.uint8)
    o.set_state(0, d.n_true, d.z, cs0, reset)
    s.set_state(0, d.n_true, torch.from_numpy(d.z), torch.from_numpy(cs0), reset)
    ls = Lockstep(f"k200-{precision}", o, s)
    ls.compare_stats()
    assert o.K > 150
    ls.iterate(4)
    ls.finish()
