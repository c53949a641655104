"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is against a value
the paper prints (the worked example of Figs. 2-3, the combination counts of
Tables 2-7), an independent library routine (scikit-learn's plug-in mutual
information, SciPy's log-likelihood G-test, numpy bincount, itertools), a
closed form (zero MI for exactly independent tables) or an invariant of the
definitions.  Mistakes such as a dropped entropy term, a wrong sign, a
transposed table or a wrong digit order in the cell index fail at least one.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.stats import chi2_contingency
from sklearn.metrics import mutual_info_score

import oracle
from paper_2201_03331_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers independent of the oracle
# --------------------------------------------------------------------------

def decode_rows(rows):
    """Genotype per sample from the 3 one-hot rows of a Fig. 2 table."""
    bits = np.array([[int(ch) for ch in r] for r in rows])
    assert (bits.sum(axis=0) == 1).all()
    return bits.argmax(axis=0)


def worked_example():
    d = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    gt = d["genotype_tables"]
    # samples 0..7 are the cases, 8..15 the controls
    a = np.concatenate([decode_rows(gt["a"]["cases"]), decode_rows(gt["a"]["controls"])])
    b = np.concatenate([decode_rows(gt["b"]["cases"]), decode_rows(gt["b"]["controls"])])
    G = np.stack([a, b]).astype(np.uint8)
    y = np.array([1] * 8 + [0] * 8, dtype=np.uint8)
    return d, G, y


def cell_labels(G, comb):
    x = np.zeros(G.shape[1], dtype=np.int64)
    for c in comb:
        x = 3 * x + G[c].astype(np.int64)
    return x


def bincount_table(G, y, comb):
    x = cell_labels(G, comb)
    k = len(comb)
    T = np.zeros((3 ** k, 2), dtype=np.int64)
    for cls in (0, 1):
        T[:, cls] = np.bincount(x[y == cls], minlength=3 ** k)
    return T


def sklearn_mi(G, y, comb):
    return mutual_info_score(cell_labels(G, comb), y.astype(np.int64))


def gtest_mi(T):
    T = np.asarray(T, dtype=np.float64)
    T = T[T.sum(axis=1) > 0]
    T = T[:, T.sum(axis=0) > 0]
    if T.shape[0] < 2 or T.shape[1] < 2:
        return 0.0
    g, _, _, _ = chi2_contingency(T, correction=False, lambda_="log-likelihood")
    return g / (2.0 * T.sum())


def random_data(rng, n, m, case_frac=0.5):
    G = rng.integers(0, 3, size=(n, m), dtype=np.uint8)
    y = (rng.random(m) < case_frac).astype(np.uint8)
    return G, y


# --------------------------------------------------------------------------
# worked example (section 3.1 Fig. 2, section 3.2 Fig. 3)
# --------------------------------------------------------------------------

def test_worked_example_tables_match_figure3():
    d, G, y = worked_example()
    exp = d["contingency_tables_cases_controls"]
    for name, comb in (("a", [0]), ("b", [1]), ("a_x_b", [0, 1])):
        T = oracle.table(G, y, comb)
        # the figure prints [cases, controls]; the tables here are [controls, cases]
        want = np.array(exp[name])[:, ::-1]
        np.testing.assert_array_equal(T, want, err_msg=name)


def test_worked_example_combined_rows_are_ands():
    """The combined table of Fig. 2 is the AND of every pairing of rows with
    the first variant outer: the cell order the oracle's index uses."""
    d, _, _ = worked_example()
    gt = d["genotype_tables"]
    for cls in ("cases", "controls"):
        for ga in range(3):
            for gb in range(3):
                ra = int(gt["a"][cls][ga], 2)
                rb = int(gt["b"][cls][gb], 2)
                assert format(ra & rb, "08b") == gt["a_x_b"][cls][3 * ga + gb]


def test_worked_example_mi_against_libraries():
    _, G, y = worked_example()
    for comb in ([0], [1], [0, 1]):
        T = oracle.table(G, y, comb)
        mi = oracle.mi(T)
        assert mi == pytest.approx(sklearn_mi(G, y, comb), rel=1e-13, abs=1e-15)
        assert mi == pytest.approx(gtest_mi(T), rel=1e-12, abs=1e-15)
    # variant b has identical case and control columns: exactly independent
    assert abs(oracle.mi(oracle.table(G, y, [1]))) <= 1e-15
    assert oracle.mi(oracle.table(G, y, [0, 1])) == pytest.approx(0.22290084190957318, rel=1e-13)
    assert oracle.mi(oracle.table(G, y, [0])) == pytest.approx(0.016911037784302615, rel=1e-13)


# --------------------------------------------------------------------------
# counting: brute force with an independent counter
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_tables_equal_bincount(k):
    rng = np.random.default_rng(100 + k)
    for n, m, frac in ((7, 1, 0.5), (8, 63, 0.3), (7, 64, 0.5), (9, 130, 0.7), (6, 200, 0.0), (6, 77, 1.0)):
        if k > n:
            continue
        G, y = random_data(rng, n, m, frac)
        for comb in itertools.combinations(range(n), k):
            np.testing.assert_array_equal(oracle.table(G, y, comb), bincount_table(G, y, comb))


def test_tables_sum_and_marginalise():
    rng = np.random.default_rng(7)
    G, y = random_data(rng, 8, 151, 0.4)
    m1 = int(y.sum())
    m0 = len(y) - m1
    for comb in itertools.combinations(range(8), 4):
        T = oracle.table(G, y, comb).astype(np.int64)
        assert T[:, 0].sum() == m0 and T[:, 1].sum() == m1
        T4 = T.reshape(3, 3, 3, 3, 2)
        for drop in range(4):
            sub = [c for i, c in enumerate(comb) if i != drop]
            want = oracle.table(G, y, sub).astype(np.int64).reshape((3,) * 3 + (2,))
            np.testing.assert_array_equal(T4.sum(axis=drop), want)


# --------------------------------------------------------------------------
# mutual information
# --------------------------------------------------------------------------

def test_mi_against_sklearn_and_gtest_random():
    rng = np.random.default_rng(11)
    for trial in range(40):
        k = int(rng.integers(1, 5))
        n = k + 2
        m = int(rng.integers(2, 600))
        G, y = random_data(rng, n, m, float(rng.uniform(0.05, 0.95)))
        comb = sorted(rng.choice(n, size=k, replace=False).tolist())
        T = oracle.table(G, y, comb)
        mi = oracle.mi(T)
        assert mi == pytest.approx(sklearn_mi(G, y, comb), rel=1e-12, abs=1e-15)
        assert mi == pytest.approx(gtest_mi(T), rel=1e-10, abs=1e-14)


def _entropy(counts):
    p = np.asarray(counts, dtype=np.float64)
    p = p[p > 0] / p.sum()
    return float(-(p * np.log(p)).sum())


def test_mi_bounds():
    rng = np.random.default_rng(12)
    for trial in range(60):
        k = int(rng.integers(1, 4))
        G, y = random_data(rng, k + 1, int(rng.integers(1, 300)), float(rng.uniform(0, 1)))
        T = oracle.table(G, y, list(range(k)))
        mi = oracle.mi(T)
        hy = _entropy(T.sum(axis=0))
        hx = _entropy(T.sum(axis=1))
        assert -1e-15 <= mi <= min(hx, hy) + 1e-15


def test_mi_invariances():
    rng = np.random.default_rng(13)
    G, y = random_data(rng, 5, 257, 0.45)
    comb = [0, 2, 3]
    base = oracle.mi(oracle.table(G, y, comb))
    # permutation of samples
    perm = rng.permutation(G.shape[1])
    assert oracle.mi(oracle.table(G[:, perm], y[perm], comb)) == pytest.approx(base, rel=1e-13, abs=1e-16)
    # swapping the class labels
    assert oracle.mi(oracle.table(G, 1 - y, comb)) == pytest.approx(base, rel=1e-13, abs=1e-16)
    # relabelling the genotype values of one variant
    G2 = G.copy()
    G2[2] = np.array([2, 0, 1], dtype=np.uint8)[G[2]]
    assert oracle.mi(oracle.table(G2, y, comb)) == pytest.approx(base, rel=1e-13, abs=1e-16)
    # the order of the variants inside the combination (rows permute)
    G3 = G[[3, 1, 0, 2, 4]]          # variants 0,2,3 now sit at 2,3,0
    T3 = oracle.table(G3, y, [0, 2, 3])
    assert oracle.mi(T3) == pytest.approx(base, rel=1e-13, abs=1e-16)


def test_mi_zero_under_duplication():
    """Every sample copied once as a control and once as a case: each cell
    holds equal counts in both classes, so MI is exactly zero in real
    arithmetic."""
    rng = np.random.default_rng(14)
    G, _ = random_data(rng, 6, 91)
    G2 = np.concatenate([G, G], axis=1)
    y2 = np.array([0] * 91 + [1] * 91, dtype=np.uint8)
    for k in (1, 2, 3):
        for comb in itertools.combinations(range(6), k):
            assert abs(oracle.mi(oracle.table(G2, y2, comb))) <= 1e-14
    # unequal copy counts (2 control copies, 1 case copy) are independent too
    G3 = np.concatenate([G, G, G], axis=1)
    y3 = np.array([0] * 182 + [1] * 91, dtype=np.uint8)
    for comb in itertools.combinations(range(6), 2):
        assert abs(oracle.mi(oracle.table(G3, y3, comb))) <= 1e-14


# --------------------------------------------------------------------------
# combination numbering
# --------------------------------------------------------------------------

def test_binom_matches_paper_tables():
    d = json.load(open(os.path.join(GOLDEN, "paper_combination_counts.json")))
    for r in d["rows"]:
        assert oracle.binom(r["variants"], r["order"]) == r["combinations"], r


def test_binom_overflow_saturates():
    assert oracle.binom(10 ** 6, 8) == 2 ** 64 - 1
    assert oracle.binom(200, 5) == math.comb(200, 5)
    assert oracle.binom(3, 5) == 0


@pytest.mark.parametrize("n,k", [(1, 1), (6, 1), (7, 3), (9, 4), (10, 5), (8, 8), (12, 6)])
def test_rank_is_lexicographic_position(n, k):
    for pos, comb in enumerate(itertools.combinations(range(n), k)):
        assert oracle.rank(n, comb) == pos
        assert oracle.unrank(n, k, pos) == comb


def test_rank_large():
    rng = np.random.default_rng(15)
    n, k = 3246, 3
    total = math.comb(n, k)
    for r in rng.integers(0, total, size=200).tolist() + [0, total - 1]:
        c = oracle.unrank(n, k, r)
        assert list(c) == sorted(set(c)) and c[-1] < n
        assert oracle.rank(n, c) == r
    assert oracle.unrank(n, k, total - 1) == (n - 3, n - 2, n - 1)


# --------------------------------------------------------------------------
# the search and its top-N
# --------------------------------------------------------------------------

def _full_sort(G, y, k):
    n = G.shape[0]
    total = math.comb(n, k)
    ranks = np.arange(total, dtype=np.uint64)
    mi = np.array([sklearn_mi(G, y, comb) for comb in itertools.combinations(range(n), k)])
    return ranks, mi


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_scan_equals_full_sort(k):
    rng = np.random.default_rng(16 + k)
    G, y = random_data(rng, 11, 150, 0.5)
    # duplicated variants give exactly tied scores; ties go to the lower rank
    G[5] = G[2]
    G[9] = G[2]
    ranks, mi_ref = _full_sort(G, y, k)
    mi_or = oracle.score_ranks(G, y, k, ranks)
    np.testing.assert_allclose(mi_or, mi_ref, rtol=1e-12, atol=1e-15)
    order = np.lexsort((ranks, -mi_or))
    for top in (1, 5, 17, len(ranks) + 3):
        for threads in (1, 3, 8):
            r, m = oracle.scan(G, y, k, top, nthreads=threads)
            want = order[: min(top, len(ranks))]
            np.testing.assert_array_equal(r, ranks[want])
            np.testing.assert_array_equal(m, mi_or[want])


def test_scan_range_pieces_merge():
    rng = np.random.default_rng(20)
    G, y = random_data(rng, 14, 97, 0.5)
    r_all, m_all = oracle.scan(G, y, 3, 25, nthreads=4)
    total = math.comb(14, 3)
    cut = 131
    r1, m1 = oracle.scan_range(G, y, 3, 25, 0, cut, nthreads=2)
    r2, m2 = oracle.scan_range(G, y, 3, 25, cut, total - cut, nthreads=5)
    r = np.concatenate([r1, r2])
    m = np.concatenate([m1, m2])
    o = np.lexsort((r, -m))[:25]
    np.testing.assert_array_equal(r[o], r_all)


def test_planted_pair_ranks_first():
    d = synth.order2_small()
    r, m = oracle.scan(d.genotypes, d.phenotype, 2, 10)
    assert oracle.unrank(d.n, 2, int(r[0])) == d.planted[0]
    assert m[0] > 3 * m[1]


def test_validate_codes():
    rng = np.random.default_rng(21)
    G, y = random_data(rng, 5, 40)
    assert oracle.validate(G, y, 2, 10) == oracle.OK
    Gb = G.copy()
    Gb[3, 7] = 3
    assert oracle.validate(Gb, y, 2, 10) == oracle.BAD_GENOTYPE
    yb = y.copy()
    yb[0] = 2
    assert oracle.validate(G, yb, 2, 10) == oracle.BAD_PHENOTYPE
    assert oracle.validate(G, y, 0, 10) == oracle.BAD_ORDER
    assert oracle.validate(G, y, 6, 10) == oracle.BAD_ORDER
    assert oracle.validate(G, y, 9, 10) == oracle.BAD_ORDER
    assert oracle.validate(G, y, 2, 0) == oracle.BAD_TOPN
