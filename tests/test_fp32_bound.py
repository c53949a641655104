"""The bound on the scan's plain single-precision MI estimate, and on the
fixed-point form of the same sum that the FP4 matrix-core kernels take.

The search filters with est = [(F(m) - F(m0)) - F(m1) + sum_x ((F(n_x0) +
F(n_x1)) - F(n_x))] * (1/m) evaluated in IEEE single precision from a float
table F of f(t) = t ln t, and keeps a combination unless est is more than
twice the bound B(k, m) = 2u (6 ln m + (3^k + 4) ln 2), u = 2^-24, below a
threshold.  Exactness of the result rests on |est - MI| <= B.  Here the same
float32 operations are replayed in numpy on random and skewed tables and
compared with the oracle's double-precision MI (itself accurate to ~1e-15).

The fixed-point form: Fq[t] = round(2^qs t ln t) modulo 2^32, qs the largest
shift with 2^qs (m ln 2 + 1) <= 2^30; D = Fq[m] - Fq[m0] - Fq[m1] + sum_x
(Fq[n_x0] + Fq[n_x1] - Fq[n_x]) modulo 2^32, read as a signed 32-bit integer,
and est = float(D) * float(2^-qs / m).  Its error is at most half a unit per
table entry (3 + 3^(k+1) entries) scaled by 2^-qs / m, plus three roundings
of the final product; the tests check that against the oracle and that it
stays below the single-precision bound above for every order up to 5.
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


def fixed_shift(m):
    span, qs = m * math.log(2.0) + 1.0, 0
    while span * 2.0 ** (qs + 1) <= 2.0 ** 30:
        qs += 1
    return qs


def table_q(m):
    qs = fixed_shift(m)
    t = np.arange(m + 1, dtype=np.float64)
    f = np.where(t > 0, t * np.log(np.maximum(t, 1)), 0.0)
    q = np.rint(np.ldexp(f, qs)).astype(np.int64)
    return (q & 0xFFFFFFFF).astype(np.uint64), qs


def estimate_fixed(T, Fq, qs):
    m0, m1 = int(T[:, 0].sum()), int(T[:, 1].sum())
    m = m0 + m1
    mask = 0xFFFFFFFF
    D = (int(Fq[m]) - int(Fq[m0]) - int(Fq[m1])) & mask
    for n0, n1 in T:
        D = (D + int(Fq[n0]) + int(Fq[n1]) - int(Fq[n0 + n1])) & mask
    if D >= 2 ** 31:
        D -= 2 ** 32
    qscale = np.float32(2.0 ** -qs / m)
    return float(np.float32(np.float32(D) * qscale))


def fixed_bound(k, m):
    u = 2.0 ** -24
    entries = 3 + 3 ** (k + 1)
    return entries * (0.5 + 2.0 ** -17) * 2.0 ** -fixed_shift(m) / m * (1 + 4 * u) + 3.0001 * u * math.log(2)


def test_fixed_point_estimate_within_bound():
    rng = np.random.default_rng(78)
    worst = 0.0
    for k in (1, 2, 3, 4, 5):
        for m in (2, 17, 1600, 6400, 8191, 20000, 100000):
            Fq, qs = table_q(m)
            B = fixed_bound(k, m)
            for trial in range(12 if k < 5 else 4):
                T = random_table(rng, k, m, skew=trial % 2 == 1)
                est = estimate_fixed(T, Fq, qs)
                mi = oracle.mi(T.astype(np.uint32))
                err = abs(est - mi)
                assert err <= B, (k, m, err, B)
                worst = max(worst, err / B)
    print("largest error / fixed-point bound:", worst)


def test_fixed_point_sum_fits_and_is_inside_the_filter_bound():
    # 2^qs m ln 2 plus the rounding of every entry stays below 2^31 (so the
    # signed reading of D is the integer sum), and the fixed-point error
    # bound is below the single-precision one the filters widen by, for
    # every class size up to 2^24 and every order up to 5
    ms = list(range(1, 4097)) + [2 ** e + d for e in range(12, 25) for d in (-1, 0, 1)]
    for m in ms:
        if m >= 2 ** 24:
            continue
        qs = fixed_shift(m)
        assert 2.0 ** qs * (m * math.log(2.0) + 1.0) <= 2.0 ** 30 < 2.0 ** (qs + 1) * (m * math.log(2.0) + 1.0)
        for k in (1, 2, 3, 4, 5):
            assert 2.0 ** qs * m * math.log(2.0) + (3 + 3 ** (k + 1)) < 2.0 ** 31
            assert fixed_bound(k, m) < bound(k, m), (k, m)

