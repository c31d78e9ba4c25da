"""Pins for the oracle's MXFP4 and MXFP6 codecs (OCP Microscaling, E2M1 and
E2M3 elements).

Sources of truth: the element values the OCP Microscaling specification prints
(the E2M1 table; the E2M3 extremes), torch's own float8 E4M3 type (E2M3 shares
its mantissa width, so its values and its rounding above 1 must agree), an
independent threshold form of round-to-nearest-even on each grid, minimality of
the power-of-two block scale, and the formats' error bounds.
"""
import numpy as np
import torch

from oracle import mx


def test_e2m1_table_is_the_specification_table():
    # OCP MX v1.0, FP4 E2M1: +-{0, 0.5, 1, 1.5, 2, 3, 4, 6}
    want = [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    t = mx.e2m1_table()
    np.testing.assert_array_equal(t[:8], want)
    np.testing.assert_array_equal(t[8:], [-v for v in want])


def _threshold_code(y):
    """Round to nearest on the E2M1 grid with ties to the even code, as a sum of
    comparisons against the midpoints (a tie at 0.25, 1.25, 2.5, 5 keeps the
    lower, even code; at 0.75, 1.75, 3.5 it takes the upper, even code)."""
    a = min(abs(float(y)), 6.0)
    m = sum(int(c) for c in (a > 0.25, a >= 0.75, a > 1.25, a >= 1.75, a > 2.5, a >= 3.5, a > 5.0))
    return m | (8 if (y < 0 and m > 0) else 0)


def test_e2m1_encode_matches_threshold_form():
    grid = mx.e2m1_table()[:8]
    mids = (grid[1:] + grid[:-1]) / 2
    rng = np.random.default_rng(0)
    ys = np.concatenate([grid, -grid, mids, -mids, np.nextafter(mids, 0), np.nextafter(mids, 10),
                         rng.uniform(-6, 6, 5000), [0.0, -0.0, 1e-30, -1e-30, 6.0, -6.0]])
    got = mx.e2m1_encode(ys)
    want = np.array([_threshold_code(y) for y in ys], np.uint8)
    np.testing.assert_array_equal(got, want)
    # every representable value encodes to itself
    np.testing.assert_array_equal(mx.e2m1_table()[mx.e2m1_encode(grid)], grid)


def test_block_exponent_is_minimal():
    rng = np.random.default_rng(1)
    for a in np.concatenate([rng.uniform(0, 1, 500) * 10.0 ** rng.integers(-30, 30, 500), [6.0, 3.0, 12.0, 1.0]]):
        e = mx.block_exponent(a)
        assert a <= 6.0 * 2.0 ** e
        assert a > 6.0 * 2.0 ** (e - 1)
    assert mx.block_exponent(0.0) == 0
    assert mx.block_exponent(1e-45) == -127                  # clamped to the E8M0 range


def test_quantize_mxfp4_error_bound_and_blocks():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((300, 128)).astype(np.float32)
    x[5, :32] *= 1e-3                                        # blocks of one row differ in scale
    x[6, 32:64] = 0.0
    codes, exps = mx.quantize_mxfp4(x)
    assert codes.shape == (300, 128) and exps.shape == (300, 4)
    assert exps[5, 0] < exps[5, 1] and exps[6, 1] == 0
    deq = mx.dequantize_mxfp4(codes, exps)
    blocks = np.abs(x.astype(np.float64)).reshape(300, 4, 32)
    s = np.ldexp(1.0, exps)
    assert (blocks.max(axis=2) <= 6.0 * s).all()
    err = np.abs(deq - x).reshape(300, 4, 32)
    # half the widest gap of the grid (between 4 and 6) is 1: |err| <= scale
    assert (err <= s[..., None]).all()
    # in the binades of the grid a nearest value is within a quarter of |x|
    y = blocks / s[..., None]
    normal = y >= 1.0
    assert (err[normal] <= 0.25 * blocks[normal] + 1e-12).all()
    np.testing.assert_array_equal(mx.dequantize_mxfp4(codes, exps)[6, 32:64], 0.0)


# --------------------------------------------------------------------- MXFP6
def _e4m3_values_torch():
    """Every finite OCP E4M3 value, decoded by torch's own float8 type."""
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    v = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    return v[np.isfinite(v)]


def test_e2m3_table_extremes_are_the_specification_values():
    # OCP MX v1.0, FP6 E2M3: max normal 7.5, min normal 1.0, max subnormal
    # 0.875, min subnormal 0.125, no infinity or NaN
    t = mx.e2m3_table()
    mags = t[:32]
    assert mags[31] == 7.5 and mags[8] == 1.0 and mags[7] == 0.875 and mags[1] == 0.125
    assert np.all(np.isfinite(t))
    assert (np.diff(mags) > 0).all()                                      # codes ordered by magnitude
    np.testing.assert_array_equal(t[32:], -mags)


def test_e2m3_values_are_the_e4m3_values_on_the_eighth_grid():
    # E2M3 has E4M3's 3 mantissa bits and a smaller exponent range: its values
    # are exactly the E4M3 values (decoded by torch) in [-7.5, 7.5] that are
    # multiples of 1/8
    e4 = _e4m3_values_torch()
    want = np.unique(e4[(np.abs(e4) <= 7.5) & (e4 * 8 == np.round(e4 * 8))])
    np.testing.assert_array_equal(np.unique(mx.e2m3_table()), want)


def _threshold_code6(y):
    """RNE on the E2M3 grid as a count of midpoints passed: between codes j and
    j + 1 a tie stays on j when j is even and moves up when j is odd."""
    grid = mx.e2m3_table()[:32]
    a = min(abs(float(y)), 7.5)
    m = 0
    for j in range(31):
        mid = (grid[j] + grid[j + 1]) / 2
        m += int(a > mid) if j % 2 == 0 else int(a >= mid)
    return m | (0x20 if (y < 0 and m > 0) else 0)


def test_e2m3_encode_matches_threshold_form_and_torch_rounding():
    grid = mx.e2m3_table()[:32]
    mids = (grid[1:] + grid[:-1]) / 2
    rng = np.random.default_rng(3)
    ys = np.concatenate([grid, -grid, mids, -mids, np.nextafter(mids, 0), np.nextafter(mids, 10),
                         rng.uniform(-7.5, 7.5, 3000), [0.0, -0.0, 1e-30, -1e-30, 7.5, -7.5]])
    got = mx.e2m3_encode(ys)
    np.testing.assert_array_equal(got, np.array([_threshold_code6(y) for y in ys], np.uint8))
    np.testing.assert_array_equal(mx.e2m3_table()[mx.e2m3_encode(grid)], grid)
    # in [1, 7.5] E2M3 and E4M3 round alike (same mantissa width, RNE): torch's cast
    f = ys.astype(np.float32)
    hi = (np.abs(f) >= 1.0) & (np.abs(f) <= 7.5)
    t = torch.from_numpy(f[hi]).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(mx.e2m3_table()[mx.e2m3_encode(f[hi].astype(np.float64))], t)
    # below 1 the grid is the fixed-point grid of step 1/8: numpy's
    # round-half-even of 8 y
    lo = np.abs(ys) < 1.0
    np.testing.assert_array_equal(np.abs(mx.e2m3_table()[mx.e2m3_encode(ys[lo])]), np.abs(np.rint(ys[lo] * 8) / 8))


def test_mxfp6_block_exponent_is_minimal():
    rng = np.random.default_rng(4)
    for a in np.concatenate([rng.uniform(0, 1, 500) * 10.0 ** rng.integers(-30, 30, 500), [7.5, 3.75, 15.0, 1.0]]):
        e = mx.block_exponent(a, 7.5)
        assert a <= 7.5 * 2.0 ** e
        assert a > 7.5 * 2.0 ** (e - 1)
    assert mx.block_exponent(7.5, 7.5) == 0 and mx.block_exponent(7.5000001, 7.5) == 1


def test_quantize_mxfp6_error_bound_and_blocks():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((300, 128)).astype(np.float32)
    x[5, :32] *= 1e-3
    x[6, 32:64] = 0.0
    codes, exps = mx.quantize_mxfp6(x)
    assert codes.shape == (300, 128) and exps.shape == (300, 4) and codes.max() < 64
    assert exps[5, 0] < exps[5, 1] and exps[6, 1] == 0
    deq = mx.dequantize_mxfp6(codes, exps)
    blocks = np.abs(x.astype(np.float64)).reshape(300, 4, 32)
    s = np.ldexp(1.0, exps)
    assert (blocks.max(axis=2) <= 7.5 * s).all()
    err = np.abs(deq - x).reshape(300, 4, 32)
    # half the widest gap of the grid (0.5, between 4 and 7.5) bounds the error
    assert (err <= 0.25 * s[..., None]).all()
    # in the binades of the grid the error is within 1/16 of |x| (3 mantissa bits)
    y = blocks / s[..., None]
    normal = y >= 1.0
    assert (err[normal] <= blocks[normal] / 16 + 1e-12).all()
    # two more mantissa bits: overall several times closer than MXFP4
    d4 = mx.dequantize_mxfp4(*mx.quantize_mxfp4(x))
    assert np.abs(deq - x).sum() * 3 < np.abs(d4 - x).sum()
