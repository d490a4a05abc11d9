"""Division by an invariant integer as the kernels do it (cell-index decode,
LDS tile addressing): m = floor(2^32 (2^L - d) / d) + 1 with L = ceil(log2 d),
n / d = (mulhi(m, n) + n) >> L for 0 <= n < 2^31 (Granlund and Montgomery,
1994).  Checked against exact integer division over divisors up to 2^24 (grid
extents are limited to 2^24 cells) and numerators spanning [0, 2^31)."""
import numpy as np


def magic(d):
    L = 0
    while (1 << L) < d:
        L += 1
    m = ((1 << 32) * ((1 << L) - d)) // d + 1
    assert 0 < m < (1 << 32)
    return m, L


def fdiv(m, L, n):
    n = n.astype(np.uint64)
    return ((((np.uint64(m) * n) >> np.uint64(32)) + n) >> np.uint64(L)).astype(np.int64)


def test_fastdiv_matches_integer_division():
    rng = np.random.default_rng(3)
    divisors = set(range(1, 520))
    for k in range(1, 25):
        divisors |= {(1 << k) - 1, 1 << k, (1 << k) + 1}
    divisors |= set(int(x) for x in rng.integers(1, 1 << 24, 100))
    top = (1 << 31) - 1
    for d in sorted(divisors):
        if d > (1 << 24):
            continue
        m, L = magic(d)
        n = np.concatenate([
            np.arange(0, 3 * d + 3, dtype=np.int64)[: 4096],
            np.array([top, top - 1, top - d, (top // d) * d, (top // d) * d - 1], dtype=np.int64),
            rng.integers(0, top, 1000, dtype=np.int64),
        ])
        n = n[(n >= 0) & (n <= top)]
        q = fdiv(m, L, n)
        assert (q == n // d).all(), d
