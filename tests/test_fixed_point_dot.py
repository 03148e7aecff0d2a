"""The integer arithmetic of the sub-cluster pass over the cluster-sorted copy
(laysub.hip, with the digit tables of layout.hip), emulated exactly in numpy
(no GPU needed).

The pass forms each cell's score difference df = sum_p x_p delta_p (eq. 8,
delta_p = log thetabar_{k,1,u} - log thetabar_{k,0,u} at place p of the
cluster's gene order, x_p <= 255 the dense counts) without floating-point
products:
  * v_p = rint(delta_p 2^E), E = 54 - e_max with |delta_p| < 2^e_max, so
    |v_p| <= 2^54;
  * v_p = sum_k d_{p,k} 256^k, seven digits in -128 .. 127;
  * the matrix cores take x - 128 as a signed byte and sum
    C_k = sum_p (x_p - 128) d_{p,k} in 32-bit integers, so that
    sum_p x_p v_p = sum_k 256^k (C_k + 128 S_k), S_k = sum_p d_{p,k};
  * df = sum_k 2^(8k - E) (C_k + 128 S_k) in FP64 (each term exact).
The statistics use the same offset: sum over the cells of a 0/1 mask times
(x - 128), plus 128 times the mask's cell count, is the exact count sum.
"""
import numpy as np

rng = np.random.default_rng(7)
PLACES = 512


def frexp_exp(d: np.ndarray) -> int:
    nz = d[d != 0]
    return int(np.frexp(np.abs(nz))[1].max()) if len(nz) else None


def digits(delta: np.ndarray):
    emax = frexp_exp(delta)
    E = 0 if emax is None else 54 - emax
    v = np.rint(np.ldexp(delta, E)).astype(np.int64)
    d = np.zeros((len(v), 8), dtype=np.int64)
    w = v.copy()
    for k in range(7):
        dk = ((w & 0xFF) ^ 0x80) - 0x80          # the low byte as a signed value
        d[:, k] = dk
        w = (w - dk) >> 8
    assert np.all(w == 0)
    return v, d, E


def cases():
    out = []
    for kind in ("normal", "wide", "tiny", "zeros", "one_big"):
        if kind == "normal":
            delta = rng.normal(0, 2.0, PLACES)
        elif kind == "wide":
            delta = rng.normal(0, 1, PLACES) * np.exp(rng.uniform(-30, 6, PLACES))
        elif kind == "tiny":
            delta = rng.normal(0, 1e-9, PLACES)
        elif kind == "zeros":
            delta = np.zeros(PLACES)
        else:
            delta = rng.normal(0, 1e-3, PLACES)
            delta[17] = -700.0
        for D in (1, 5, 8):
            x = rng.integers(0, 256, size=(64, 64 * D))
            x[rng.random(x.shape) < 0.8] = 0
            x[:, :3] = 255                               # the largest bytes
            out.append((delta, D, x))
    return out


def test_digits_reconstruct_the_fixed_point_values():
    for delta, _, _ in cases():
        v, d, _ = digits(delta)
        assert np.all(np.abs(v) <= 2 ** 54)
        assert np.all((d >= -128) & (d <= 127))
        assert np.all(d[:, 7] == 0)
        recon = np.zeros(len(v), dtype=object)
        for k in range(7):
            recon = recon + d[:, k].astype(object) * (256 ** k)
        assert np.all(recon == v.astype(object))


def test_offset_digit_sums_give_the_exact_integer_dot():
    for delta, D, x in cases():
        v, d, E = digits(delta)
        n = 64 * D
        dd = d[:n]
        S = dd.sum(axis=0)
        xs = x - 128                                      # signed bytes
        assert xs.min() >= -128 and xs.max() <= 127
        C = xs @ dd                                       # what the matrix cores sum, per cell and digit
        assert np.abs(C).max() < 2 ** 31 and np.abs(C + 128 * S).max() < 2 ** 53
        exact = (x.astype(object) @ v[:n].astype(object))
        via = np.zeros(len(x), dtype=object)
        for k in range(8):
            via = via + (C[:, k] + 128 * S[k]).astype(object) * (256 ** k)
        assert np.all(via == exact)


def test_fp64_result_within_the_fixed_point_rounding():
    """In exact arithmetic |2^-E sum x v - sum x delta| <= 2^(-E-1) sum x
    (each v_p is delta_p 2^E rounded to an integer), and the kernel's FP64
    sum of the eight exact terms is within 8 units of 2^-53 of the
    fixed-point value."""
    from fractions import Fraction
    for delta, D, x in cases():
        v, d, E = digits(delta)
        n = 64 * D
        C = (x - 128) @ d[:n]
        S = d[:n].sum(axis=0)
        df = np.zeros(len(x))
        for k in range(8):
            df = df + np.ldexp((C[:, k] + 128 * S[k]).astype(np.float64), 8 * k - E)
        for row in range(0, len(x), 16):
            xs = [int(t) for t in x[row]]
            assert E >= 0                                 # |delta| < 2^54 in every case here
            fixed = Fraction(sum(a * int(b) for a, b in zip(xs, v[:n])), 2 ** E)
            true = sum(Fraction(a) * Fraction(float(b)) for a, b in zip(xs, delta[:n]))
            assert abs(fixed - true) <= Fraction(sum(xs), 2 ** (E + 1))
            assert abs(Fraction(float(df[row])) - fixed) <= 8 * 2.0 ** -53 * abs(fixed) + Fraction(1, 2 ** 1074)


def test_statistics_offset_identity():
    """sum_c m_c (x_c - 128) + 128 sum_c m_c = sum_c m_c x_c for 0/1 masks
    over a wavefront's 32 cells (all within 32-bit integers)."""
    x = rng.integers(0, 256, size=(32, 64))
    for _ in range(20):
        m = (rng.random((4, 32)) < 0.5).astype(np.int64)
        o = m @ (x - 128)
        assert np.abs(o).max() <= 32 * 128
        assert np.array_equal(o + 128 * m.sum(axis=1)[:, None], m @ x)
