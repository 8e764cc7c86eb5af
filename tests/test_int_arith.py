"""Host-side checks of the integer shortcuts the kernels take (the kernels run
them on the GPU; the arithmetic they rely on is checked here exhaustively or on
dense samples).

* Division by a mesh or branch divisor d through m = floor((2^32 - 1) / d): the
  high product x m / 2^32 is floor(x / d) or one less for every 32-bit x, so one
  remainder test gives the quotient.
* Reduction mod n by compare-and-subtract folds, exact for x in (-4n, 4n).
"""
import numpy as np


def udivm(x, d, m):
    q = (x * m) >> 32
    return q + 1 if x - q * d >= d else q


def wrapn(x, n):
    x = x + 2 * n if x < 0 else x
    x = x + 2 * n if x < 0 else x
    x = x - 2 * n if x >= 2 * n else x
    return x - n if x >= n else x


def test_division_by_inverse():
    rng = np.random.default_rng(5)
    for d in list(range(1, 1025)) + [1 << 16, 4096 * 4096 - 1, 12345678]:
        m = (2**32 - 1) // d
        xs = set(int(v) for v in rng.integers(0, 2**32, size=400))
        xs |= {0, 1, d - 1, d, d + 1, 2**32 - 1, 2**32 - 2, (2**32 - 1) // d * d, (2**32 - 1) // d * d - 1}
        for k in range(1, 50):  # around multiples of d
            for x in (k * d - 1, k * d, k * d + 1):
                if 0 <= x < 2**32:
                    xs.add(x)
        for x in xs:
            q0 = (x * m) >> 32
            assert q0 in (x // d, x // d - 1), (x, d)
            assert udivm(x, d, m) == x // d, (x, d)


def test_division_small_exhaustive():
    # every x below 2^16 for the divisors of meshes up to 64 and two-to-eight-atom cells
    xs = np.arange(1 << 16, dtype=np.uint64)
    for d in list(range(1, 65)) + [96, 576, 4096]:
        m = np.uint64((2**32 - 1) // d)
        q = (xs * m) >> np.uint64(32)
        q = np.where(xs - q * np.uint64(d) >= d, q + np.uint64(1), q)
        assert np.array_equal(q, xs // np.uint64(d)), d


def test_mod_folds():
    for n in (1, 2, 3, 7, 8, 10, 16, 33, 64, 1024):
        for x in range(-4 * n + 1, 4 * n):
            assert wrapn(x, n) == x % n, (x, n)
