"""Pins for the oracle's MXFP4 codec (OCP Microscaling, E2M1 elements).

Sources of truth: the E2M1 value table printed in the OCP Microscaling
specification, an independent threshold form of round-to-nearest-even on that
grid, minimality of the power-of-two block scale, and the format's error bound.
"""
import numpy as np

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
