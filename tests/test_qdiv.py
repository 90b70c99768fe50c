"""The exact small-integer quotient used by the general LDS transforms'
index arithmetic (QDiv in the device header): t / d = trunc(t * r) with
r = fl(fl(1/d) * (1 + 1.5 * 2^-20)), all in IEEE binary32 with round to
nearest.  Emulated here with numpy float32 (the same correctly rounded
operations the kernels use: a full-precision divide and two multiplies) and
checked against integer division over every (t, d) the transforms can form
at their tile sizes, plus the range bound t < 2^19 the header states."""

import numpy as np

RAISE = np.float32(1.0 + 1.5 * 2.0 ** -20)


def qquo(t, d):
    r = (np.float32(1.0) / np.float32(d)) * RAISE
    return (t.astype(np.float32) * r).astype(np.int64)


def test_raise_constant_is_exact():
    assert float(RAISE) == 1.0 + 1.5 * 2.0 ** -20


def test_every_tile_quotient():
    t = np.arange(1 << 14, dtype=np.int64)   # offsets within the largest LDS tile
    for d in range(1, 4097):
        np.testing.assert_array_equal(qquo(t, d), t // d, err_msg=f"d={d}")


def test_range_bound():
    rng = np.random.default_rng(0)
    t = np.concatenate([np.arange((1 << 19) - 4096, 1 << 19), rng.integers(0, 1 << 19, 1 << 16)])
    t = t.astype(np.int64)
    for d in list(range(1, 300)) + [int(x) for x in rng.integers(300, 1 << 18, 400)]:
        # multiples of d and their neighbours are the critical points
        m = np.arange(0, (1 << 19) // d + 1, dtype=np.int64) * d
        tt = np.concatenate([t, m, np.maximum(m - 1, 0)])
        tt = tt[tt < (1 << 19)]
        np.testing.assert_array_equal(qquo(tt, d), tt // d, err_msg=f"d={d}")
