"""The bound on the scan's plain single-precision MI estimate.

The search filters with est = [(F(m) - F(m0)) - F(m1) + sum_x ((F(n_x0) +
F(n_x1)) - F(n_x))] * (1/m) evaluated in IEEE single precision from a float
table F of f(t) = t ln t, and keeps a combination unless est is more than
twice the bound B(k, m) = 2u (6 ln m + (3^k + 4) ln 2), u = 2^-24, below a
threshold.  Exactness of the result rests on |est - MI| <= B.  Here the same
float32 operations are replayed in numpy on random and skewed tables and
compared with the oracle's double-precision MI (itself accurate to ~1e-15).
"""
import math

import numpy as np

import oracle


def bound(k, m):
    u = 2.0 ** -24
    return 2 * u * (6 * math.log(m) + (3 ** k + 4) * math.log(2))


def estimate(T, F):
    m0, m1 = int(T[:, 0].sum()), int(T[:, 1].sum())
    m = m0 + m1
    f32 = np.float32
    s = f32(f32(F[m] - F[m0]) - F[m1])
    for n0, n1 in T:
        s = f32(s + f32(f32(F[n0] + F[n1]) - F[n0 + n1]))
    return float(f32(s * f32(f32(1.0) / f32(m))))


def table_f(m):
    t = np.arange(m + 1, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(t > 0, t * np.log(np.maximum(t, 1)), 0.0)
    return f.astype(np.float32)


def random_table(rng, k, m, skew):
    cells = 3 ** k
    if skew:
        p = rng.dirichlet(np.full(cells * 2, 0.05))
    else:
        p = rng.dirichlet(np.full(cells * 2, 5.0))
    counts = rng.multinomial(m, p).reshape(cells, 2)
    return counts.astype(np.int64)


def test_estimate_within_bound():
    rng = np.random.default_rng(77)
    worst = 0.0
    for k in (1, 2, 3, 4, 5):
        for m in (2, 17, 1600, 6400, 20000, 100000):
            F = table_f(m)
            B = bound(k, m)
            for trial in range(12 if k < 5 else 4):
                T = random_table(rng, k, m, skew=trial % 2 == 1)
                est = estimate(T, F)
                mi = oracle.mi(T.astype(np.uint32))
                err = abs(est - mi)
                assert err <= B, (k, m, err, B)
                worst = max(worst, err / B)
    print("largest error / bound:", worst)


def test_bound_values_used_by_the_workloads():
    # the filter margin 2B relative to typical cut-off scores of the workloads
    assert bound(3, 6400) < 1e-5
    assert bound(2, 16000) < 1e-5
    assert bound(5, 4000) < 3e-5
