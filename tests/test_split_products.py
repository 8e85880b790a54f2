"""The arithmetic of the split-product flush, checked on the host by exact
emulation: an FP32 value x split into three BF16 parts (x0 the nearest BF16 to
x, x1 to x - x0, x2 to x - x0 - x1, each difference exact in FP32) leaves at
most u^3 |x| = 2^-24 |x| (u = 2^-8, the unit roundoff of BF16), and the sum of
the six part products a_i b_j with i + j <= 2 (each exact in FP32) differs from
a b by at most 4 u^3 |a||b|: a few units of FP32 rounding, the accuracy the
flush claims for its FP32 products."""
import numpy as np

U = 2.0 ** -8


def bf16_rn(x):
    """Nearest BF16 (ties to even) of float32 values, returned as float32."""
    x = np.asarray(x, np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split3(x):
    x = np.asarray(x, np.float32)
    x0 = bf16_rn(x)
    r1 = (x - x0).astype(np.float32)
    x1 = bf16_rn(r1)
    x2 = bf16_rn((r1 - x1).astype(np.float32))
    return x0, x1, x2


def _values(n, seed):
    rng = np.random.default_rng(seed)
    mag = np.exp2(rng.uniform(-60.0, 60.0, n))
    x = (rng.uniform(1.0, 2.0, n) * mag * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    # values that sit exactly on BF16 rounding boundaries and plain BF16 values
    edge = np.array([1.0, -1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9,
                     1.0 - 2.0 ** -24, 2.0 ** -100, 3.0e38, 0.0], np.float32)
    return np.concatenate([x, edge])


def test_three_parts_leave_at_most_u3():
    x = _values(200000, 0)
    x0, x1, x2 = split3(x)
    xd = x.astype(np.float64)
    res = np.abs(xd - x0.astype(np.float64) - x1.astype(np.float64) - x2.astype(np.float64))
    assert np.all(res <= U ** 3 * np.abs(xd))
    # the differences the split forms are exact in FP32
    assert np.all((x.astype(np.float64) - x0) == (x - x0).astype(np.float64))
    assert np.all(np.abs(x1.astype(np.float64)) <= U * np.abs(xd))
    assert np.all(np.abs(x2.astype(np.float64)) <= U * U * np.abs(xd) * (1 + U))


def test_six_part_products_within_4u3():
    a = _values(100000, 1)
    b = _values(100000, 2)
    # keep the exact products within FP32 range, away from underflow
    ok = (np.abs(a.astype(np.float64) * b) < 1e30) & (np.abs(a.astype(np.float64) * b) > 1e-30)
    a, b = a[ok], b[ok]
    pa, pb = split3(a), split3(b)
    s = np.zeros(a.shape, np.float64)
    for i in range(3):
        for j in range(3 - i):
            # each part product is exact in FP32 (8 + 8 significant bits)
            prod32 = (pa[i] * pb[j]).astype(np.float64)
            assert np.all(prod32 == pa[i].astype(np.float64) * pb[j].astype(np.float64))
            s += prod32
    exact = a.astype(np.float64) * b.astype(np.float64)
    assert np.all(np.abs(s - exact) <= 4 * U ** 3 * np.abs(exact))


def test_a_dropped_term_or_part_breaks_the_bound():
    """Planted mistakes fail the bound: two parts only, or the i + j = 2 products
    dropped, leave errors of order u^2 |a||b|, far above 4 u^3."""
    a = _values(20000, 3)
    b = _values(20000, 4)
    ok = (np.abs(a.astype(np.float64) * b) < 1e30) & (np.abs(a.astype(np.float64) * b) > 1e-30)
    a, b = a[ok], b[ok]
    pa, pb = split3(a), split3(b)
    exact = a.astype(np.float64) * b.astype(np.float64)
    s = sum((pa[i] * pb[j]).astype(np.float64) for i in range(2) for j in range(2 - i))
    assert np.max(np.abs(s - exact) / np.abs(exact)) > 16 * U ** 3
    x0, x1 = pa[0], pa[1]
    res = np.abs(a.astype(np.float64) - x0 - x1.astype(np.float64))
    assert np.max(res / np.abs(a.astype(np.float64))) > 4 * U ** 3
