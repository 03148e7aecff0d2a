"""The certified rounding bound of the split-BF16 cluster scores, pinned by a
worst-case emulation on the CPU (no GPU needed).

The matrix-core kernel (assign_mfma.hip) scores a cell with n non-zero counts
as S = sum over its dense entries of x (hi + lo) (BF16 hi/lo of FP32 log theta,
products exact; a count above 255 on one of the first 32 places of the block's
cluster is split into its low byte and 256 x its high byte, four exact
products, and counted as two entries) plus sum over its tail entries of
fp32(x fp32(log theta)), all added in FP32, then adds log pi and the Gumbel
noise.  The kernel trusts a
decision when the gap of its two best values exceeds the sum of their bounds
    b(S, lp, n) = (2^-17 + (2n + 8) 2^-23) 1.01 (|S| + |lp| + 20) + 1e-5,
evaluated in FP32 on its own S.  The hardware assumption is that each FP32
addition of two non-zero values errs by at most one unit in the last place of
its result and that adding a zero is exact, in whatever order the matrix cores
sum.  The emulation takes the worst case of that assumption: all terms have
the same sign, they are added largest first (the largest partial sums), and
every addition rounds in the same direction (toward -inf or toward zero, error
below one ulp), with the encode exactly as the redraw kernel does it.  The FP64
reference uses the FP64 log theta.  Every case must satisfy
|S_emul - S_exact| <= b.  Two constructed cases show that the bound's terms are
needed: one where the hi and the lo product of every entry each lose almost an
ulp (so a bound counting one addition per entry fails), and one whose error is
all in the hi/lo representation (so a bound without the 2^-17 term fails).
"""
import numpy as np

rng = np.random.default_rng(2024)


def bf16_rne(f32: np.ndarray) -> np.ndarray:
    """float32 -> the nearest BF16 value (ties to even), as float64."""
    b = np.asarray(f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f32(v: float, mode: str) -> np.float32:
    """v rounded to float32 toward -inf ("down") or toward zero ("zero"),
    error below one ulp."""
    f = np.float32(v)
    if mode == "down" and float(f) > v:
        f = np.nextafter(f, np.float32(-np.inf))
    elif mode == "zero" and abs(float(f)) > abs(v):
        f = np.nextafter(f, np.float32(0.0))
    return f


def emulate(x: np.ndarray, lt: np.ndarray, dense: np.ndarray, lp: float, gumbel: float, mode: str = "down",
            split: np.ndarray = None):
    """Worst-case FP32 score of one cell: x counts, lt FP64 log theta of its
    genes, dense[i] whether entry i is in the dense chunks (x <= 255), split[i]
    whether a count above 255 is split into its low byte (a dense chunk) and
    256 x its high byte (the high plane): four products, each exact."""
    f = lt.astype(np.float32)
    hi = bf16_rne(f)
    lo = bf16_rne((lt - hi).astype(np.float32))
    if split is None:
        split = np.zeros(len(x), dtype=bool)
    terms = []
    for xi, fi, hi_i, lo_i, d, s in zip(x, f, hi, lo, dense, split):
        if s:
            lb, hb = xi % 256.0, xi - xi % 256.0       # 256 x the high byte: 8 significant bits
            terms += [lb * hi_i, lb * lo_i, hb * hi_i, hb * lo_i]
        elif d:
            terms += [xi * hi_i, xi * lo_i]          # exact in FP32 (8-bit x 8-bit significands)
        else:
            terms.append(float(round_f32(float(xi) * float(fi), mode)))
    terms = sorted(terms, key=abs, reverse=True)
    acc = np.float32(0.0)
    for tm in terms:
        if tm == 0.0:
            continue                                  # adding a zero is exact
        acc = round_f32(float(acc) + tm, mode)
    score = acc
    val = round_f32(float(round_f32(float(score) + lp, mode)) + gumbel, mode)
    exact_score = float(np.sum(x * lt))
    return float(score), float(val), exact_score


def bound(S: float, lp: float, n: int, adds_per_entry: int = 2, repr_term: bool = True) -> float:
    f32 = np.float32
    fac = (f32(2.0 ** -17 if repr_term else 0.0) + f32(adds_per_entry * n + 8) * f32(2.0 ** -23)) * f32(1.01)
    return float(fac * (f32(abs(S)) + f32(abs(lp)) + f32(20.0)) + f32(1e-5))


def cases():
    """(x, log theta, dense flags, log pi, gumbel): long rows, extreme log theta."""
    out = []
    for n in (1, 7, 64, 512, 2000, 4000):
        for kind in ("uniform", "extreme", "big_counts", "tail_heavy"):
            if kind == "uniform":
                x = rng.integers(1, 256, size=n)
                lt = np.log(rng.dirichlet(np.ones(n)) + 1e-300)
            elif kind == "extreme":
                x = rng.integers(1, 256, size=n)
                lt = -np.exp(rng.uniform(np.log(1e-6), np.log(60.0), size=n))
            elif kind == "big_counts":
                x = rng.integers(1, 65536, size=n)
                lt = -rng.uniform(1e-4, 40.0, size=n)
            else:
                x = rng.integers(1, 4000, size=n)
                lt = -rng.uniform(0.5, 25.0, size=n)
            dense = (x <= 255) & (rng.random(n) < 0.8)
            out.append((x.astype(np.float64), lt, dense, float(-rng.uniform(0, 30)), float(rng.uniform(-2.8, 16.6))))
    return out


def test_bound_dominates_worst_case_rounding():
    worst = 0.0
    for mode in ("down", "zero"):
        for x, lt, dense, lp, g in cases():
            S, val, exact = emulate(x, lt, dense, lp, g, mode)
            b = bound(S, lp, len(x))
            # the score alone and the value with log pi and noise (up to the
            # noise's own FP32 error, which the 1e-5 covers)
            assert abs(S - exact) <= b, (mode, len(x), S, exact, b)
            assert abs(val - (exact + lp + g)) <= b, (mode, len(x), val, exact + lp + g, b)
            worst = max(worst, abs(S - exact) / b)
    assert worst > 0.1, worst


def test_bound_covers_split_counts():
    """Counts above 255 split between a dense chunk and the high plane: the
    kernel counts each as two entries (lay_nnz), so a cell with n entries of
    which s are split is bounded with n + s."""
    worst = 0.0
    for mode in ("down", "zero"):
        for x, lt, dense, lp, g in cases():
            split = (x >= 256) & (rng.random(len(x)) < 0.6)
            S, val, exact = emulate(x, lt, dense, lp, g, mode, split)
            b = bound(S, lp, len(x) + int(split.sum()))
            assert abs(S - exact) <= b, (mode, len(x), S, exact, b)
            assert abs(val - (exact + lp + g)) <= b
            worst = max(worst, abs(S - exact) / b)
    assert worst > 0.1, worst


def adversarial_two_ulps(m: int):
    """A tail entry whose product is about -2^24 (ulp 2), then m dense entries
    x = 255, log theta = -4.0390625 = hi + lo exactly (hi = -4.03125,
    lo = -2^-7): each adds x hi = -1027.97 and x lo = -1.99, and rounding
    toward zero loses 1.97 + 1.99, almost two ulps, per entry."""
    x = np.r_[65535.0, np.full(m, 255.0)]
    lt = np.r_[-257.0, np.full(m, -4.0390625)]
    dense = np.r_[False, np.ones(m, dtype=bool)]
    return x, lt, dense


def test_two_inexact_additions_per_entry_are_needed():
    for m in (512, 2000, 4000):
        x, lt, dense = adversarial_two_ulps(m)
        S, _, exact = emulate(x, lt, dense, 0.0, 0.0, "zero")
        err = abs(S - exact)
        assert err > 3.9 * m                                   # about two ulps (2 each) per entry
        assert err <= bound(S, 0.0, len(x))
        assert err > bound(S, 0.0, len(x), adds_per_entry=1)


def test_representation_term_is_needed():
    """One entry of x = 255 whose log theta has a hi/lo residual near 2^-18
    relative: the products and the single addition are exact, so the whole
    error is the representation, which only the 2^-17 term covers."""
    lt = -np.exp(rng.uniform(np.log(20.0), np.log(80.0), size=200000))
    hi = bf16_rne(lt.astype(np.float32))
    lo = bf16_rne((lt - hi).astype(np.float32))
    j = int(np.argmax(np.abs(lt - hi - lo) / np.abs(lt)))
    x, l1 = np.array([255.0]), lt[j: j + 1]
    S, _, exact = emulate(x, l1, np.array([True]), 0.0, 0.0)
    assert abs(S - exact) <= bound(S, 0.0, 1)
    assert abs(S - exact) > bound(S, 0.0, 1, repr_term=False)


def test_encode_residual():
    """|log theta - hi - lo| <= 2^-17 |log theta| for the encode above."""
    lt = -np.exp(rng.uniform(np.log(1e-8), np.log(80.0), size=200000))
    f = lt.astype(np.float32)
    hi = bf16_rne(f)
    lo = bf16_rne((lt - hi).astype(np.float32))
    assert np.all(np.abs(lt - hi - lo) <= 2.0 ** -17 * np.abs(lt))
