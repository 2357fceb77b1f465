"""Host checks of arithmetic identities the kernels rely on (no GPU): the small-operand division
through the FP32 hardware reciprocal (floor((a + 1/2) * rcp(b)) == a // b for a < 2^16, b <= 128,
with the reciprocal anywhere within 1 ulp of 1/b, as the hardware instruction guarantees), and
the exact integer sums of the half-shell pair kernel's partner terms (modular uint64 arithmetic:
wrap-around is intended)."""
import numpy as np
import pytest


def test_small_division_through_fp32_reciprocal():
    a = np.arange(0, 1 << 16, dtype=np.int64)
    af = a.astype(np.float32) + np.float32(0.5)
    for b in range(1, 129):
        r = np.float32(1.0) / np.float32(b)
        for rb in (np.nextafter(r, np.float32(0)), r, np.nextafter(r, np.float32(np.inf))):
            q = (af * rb).astype(np.int64)  # FP32 product, then truncation toward zero
            np.testing.assert_array_equal(q, a // b)


# ---------------------------------------------------------------- exact partner sums
# The half-shell pair kernel adds partner terms as 64-bit integers: the bit pattern of x + M,
# M = 1.5 * 2^52, is that of M plus round(x) (|x| < 2^51), and the residual x - round(x) is exact.
# Below the same steps in numpy FP64 / uint64 arithmetic, checked against exact rational sums.
from fractions import Fraction

M = 6755399441055744.0
MBITS = np.float64(M).view(np.uint64)


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def _terms(n, scale, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) * scale * rng.choice([1e-6, 1e-2, 1.0, 1e3], size=n)


def test_magic_constant_rounds_to_integer_and_residual_is_exact():
    x = np.concatenate([_terms(4000, 1e4, 1), np.array([0.5, -0.5, 1.5, 2.5, -2.5, 2.0 ** 50 - 0.5, -(2.0 ** 50)])])
    a = x + M
    h = a - M
    np.testing.assert_array_equal(h, np.rint(x))  # round half to even
    np.testing.assert_array_equal((_bits(a) - MBITS).view(np.int64), np.rint(x).astype(np.int64))
    r = x - h
    for xi, hi, ri in zip(x, h, r):
        assert Fraction(ri) == Fraction(xi) - Fraction(hi)  # the residual is exact
    assert np.all(np.abs(r) <= 0.5)


def _fx_sum(x):
    """fx_add / fx_value: 64-bit words of round(x) and round((x - round(x)) 2^50)."""
    a = x + M
    h = a - M
    b = (x - h) * 2.0 ** 50 + M  # the kernel uses one fma; x - h is exact and the scaling too
    k = np.uint64(len(x))
    with np.errstate(over="ignore"):
        hi = (np.sum(_bits(a), dtype=np.uint64) - k * MBITS).view(np.int64)
        lo = (np.sum(_bits(b), dtype=np.uint64) - k * MBITS).view(np.int64)
    return int(hi), int(lo)


def test_two_word_sum_is_order_free_and_within_its_resolution():
    for seed in range(5):
        x = _terms(256, 1e3, 10 + seed)
        hi, lo = _fx_sum(x)
        hi2, lo2 = _fx_sum(x[np.random.default_rng(seed).permutation(len(x))])
        assert (hi, lo) == (hi2, lo2)  # integer sums: any order gives the same words
        exact = sum(Fraction(v) for v in x)
        got = Fraction(hi) + Fraction(lo, 2 ** 50)
        assert abs(got - exact) <= Fraction(len(x), 2 ** 51)  # each residual rounded to 2^-50


def test_one_word_sum_resolution():
    """fx1_add / fx1_value (FP32 path): round(x 2^26) in one word, |x| < 2^24."""
    for seed in range(5):
        x = _terms(256, 1e2, 20 + seed)
        assert np.all(np.abs(x) < 2.0 ** 24)
        with np.errstate(over="ignore"):
            w = (np.sum(_bits(x * 2.0 ** 26 + M), dtype=np.uint64) - np.uint64(len(x)) * MBITS).view(np.int64)
        exact = sum(Fraction(v) for v in x)
        assert abs(Fraction(int(w), 2 ** 26) - exact) <= Fraction(len(x), 2 ** 27)


def test_two_word_sum_with_32_bit_high_word():
    """fx2_add (FP64 path): round(x) from the low half of the bit pattern of x + M, summed in 32
    bits (|x| < 2^23 and at most 256 terms cannot overflow it)."""
    x = _terms(256, 1e4, 30)
    x[0], x[1] = 2.0 ** 23 - 1.0, -(2.0 ** 23 - 1.0)
    low = (_bits(x + M) & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32).astype(np.int64)
    np.testing.assert_array_equal(low, np.rint(x).astype(np.int64))
    assert abs(int(low.sum())) < 2 ** 31


# ---------------------------------------------------------------- FP32 cutoff test of the LJ kernel
# The single-site pair kernel lists candidate j for molecule i when
#   T = fma(-2 z~_i, z~_j, fma(-2 y~_i, y~_j, fma(-2 x~_i, x~_j, n~_j))) < fl32(thr - n~_i),
# x~ = fl32(x - o) relative to the tile centre o, n~ = fma(z~, z~, fma(y~, y~, x~ * x~)) in FP32,
# and decides exactly in FP64 afterwards.  The threshold below (the kernel's bound, restated)
# must let every pair with FP64 r^2 < r_c^2 through.  Emulation: FP32 values held in float64,
# each FMA as the exact product plus the addend rounded once to float64, then once to float32
# (the float64 step can differ from a fused FP32 FMA by a rounding of 2^-53 relative, far below
# the margins measured here).

def _guard_threshold(rc, hx, hy, hz):
    u = 2.0 ** -24
    R = np.sqrt(2.25 * hx * hx + 4.0 * hy * hy + 4.0 * hz * hz) * (1.0 + 1e-12)
    thr = (rc * rc + 4.0 * u * R * rc + 17.0 * u * R * R) * (1.0 + 2.0 * u)
    t = np.float32(thr)
    if float(t) < thr:
        t = np.nextafter(t, np.float32(np.inf))
    return t


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _fma32(a, b, c):
    return _f32(a * b + c)


@pytest.mark.parametrize("rc,h", [(2.5, 2.5413249), (3.0, 3.0097), (2.5, 2.8499600), (2.5, 3.7), (6.0, 6.2)])
def test_fp32_cutoff_threshold_never_drops_a_pair(rc, h):
    rng = np.random.default_rng(int(rc * 1000 + h * 10))
    n = 200000
    thr = float(_guard_threshold(rc, h, h, h))
    o = rng.uniform(0.0, 50.0, size=3)
    # i anywhere in the tile's home region, j at a distance just inside (or at) the cutoff in a
    # random direction, clipped to the staged extent (1.5 h in x, 2 h in y and z from o)
    ext = np.array([1.5 * h, 2.0 * h, 2.0 * h])
    xi = o + rng.uniform(-0.5, 0.5, size=(n, 3)) * np.array([h, 2 * h, 2 * h])
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = rc * (1.0 - rng.uniform(0.0, 1e-6, size=n) * rng.choice([1e-9, 1e-6, 1e-3, 1.0], size=(n,)))
    xj = xi - r[:, None] * v
    keep = np.all(np.abs(xj - o) <= ext, axis=1)
    xi, xj = xi[keep], xj[keep]
    d = xi - xj
    r2 = d[:, 2] * d[:, 2] + (d[:, 1] * d[:, 1] + d[:, 0] * d[:, 0])  # near-exact; ties decided below
    inside = r2 < rc * rc
    a, b = _f32(xi - o), _f32(xj - o)
    nj = _fma32(b[:, 2], b[:, 2], _fma32(b[:, 1], b[:, 1], _f32(b[:, 0] * b[:, 0])))
    ni = _fma32(a[:, 2], a[:, 2], _fma32(a[:, 1], a[:, 1], _f32(a[:, 0] * a[:, 0])))
    T = _fma32(-2.0 * a[:, 2], b[:, 2], _fma32(-2.0 * a[:, 1], b[:, 1], _fma32(-2.0 * a[:, 0], b[:, 0], nj)))
    thri = _f32(thr - ni)
    assert inside.sum() > 1000
    margin = (thri - T)[inside]
    assert np.all(margin > 0.0), f"a pair inside the cutoff fails the FP32 test (min margin {margin.min()})"
    # the threshold stays close to r_c^2: few extra pairs reach the exact test
    assert thr / (rc * rc) - 1.0 < 1e-4
