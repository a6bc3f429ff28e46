"""The arithmetic behind the parity step (host only).

The FP32 grid kernels take Eq. (4)'s sign from the parity of floor(2d),
d = x_u - x_v, read off the lowest mantissa bit of 1.5 * 2^23 + floor(2d) (an
fma rounded toward minus infinity), and flip the sign bit of alpha J by that bit.
Checked here without a GPU: the decision equals fract(d) < 1/2 for every d the
grid can produce (dense samples, and every exact tie at 0, 1/2, 1 and one grid
step either side), the lowest bit of 1.5 * 2^23 + k is the parity of k for the
integers the kernels meet, and adding that bit shifted to bit 31 to the bits of
alpha J negates it exactly when the bit is set."""
import numpy as np

STEP = 2.0 ** -23
MAGIC = np.float32(1.5 * 2.0 ** 23)


def parity_sign(d):
    """The kernels' decision: +1 when floor(2d) is even."""
    k = np.floor(2.0 * np.asarray(d, dtype=np.float64)).astype(np.int64)
    return np.where(k % 2 == 0, 1, -1)


def fract_sign(d):
    """Eq. (4)'s decision as the oracle takes it: +1 when fract(d) < 1/2."""
    d = np.asarray(d, dtype=np.float64)
    return np.where(d - np.floor(d) < 0.5, 1, -1)


def test_parity_equals_fract_rule_on_the_grid():
    rng = np.random.default_rng(5)
    # differences of grid phases in the lazy range (-1/2, 3/2): |d| < 2
    k = rng.integers(-(2 ** 24) + 1, 2 ** 24, size=200_000)
    d = k * STEP
    assert np.array_equal(parity_sign(d), fract_sign(d))
    ties = np.array([t + e * STEP for t in (-1.5, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5)
                     for e in (-1, 0, 1)])
    assert np.array_equal(parity_sign(ties), fract_sign(ties))
    # the two decisions at the ties themselves: 0 and 1 count +1, 1/2 counts -1
    assert list(parity_sign(np.array([0.0, 1.0, -1.0, 0.5, -0.5, 1.5]))) == [1, 1, 1, -1, -1, -1]


def test_lowest_mantissa_bit_is_the_parity():
    # 2d lies in (-4, 4): the fma result 1.5 * 2^23 + floor(2d) is an integer in
    # [2^23, 2^24), where FP32 has unit spacing
    for kk in range(-4, 5):
        v = np.float32(MAGIC + np.float32(kk))
        assert float(v) == 1.5 * 2.0 ** 23 + kk
        assert (int(v.view(np.uint32)) & 1) == (kk & 1)


def test_sign_flip_by_adding_the_bit():
    rng = np.random.default_rng(6)
    aj = (rng.integers(1, 2 ** 22, size=1000) * 2.0 ** -22).astype(np.float32)
    aj[::2] *= -1  # J of either sign
    bits = aj.view(np.uint32).astype(np.uint64)
    for p in (0, 1):
        out = ((bits + (p << 31)) & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
        assert np.array_equal(out, aj if p == 0 else -aj)
