"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: contingency tables and the top-N set (ranks, order) bit-exact; the FP64
score of every hit bit-identical to the oracle's (same table, same Eq. 1-3
evaluation order); the compensated FP32 score within 1e-5 relative + 1e-10
absolute of the FP64 one; the counting kernel's own plain FP32 estimate of
every hit (fiuncho_hit.est, computed from the kernel's counts) within the
rounding bound fiuncho_estimate_bound of the oracle's MI -- one miscounted
cell moves MI by about ln(2)/m, far more than that bound.  The full-size
workloads are compared with a complete oracle scan.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2201_03331_amd import fiuncho, synth

pytestmark = pytest.mark.gpu

TOL_REL = 1e-5
TOL_ABS = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_est(hits, k, m, mi_ref=None):
    """The counting kernel's estimate of every hit lies within the stated
    bound of the exact MI (the oracle's, when given)."""
    if len(hits) == 0:
        return
    ref = hits["mi"] if mi_ref is None else mi_ref
    bound = fiuncho.estimate_bound(k, m)
    d = np.abs(hits["est"].astype(np.float64) - ref)
    assert np.all(d <= bound), (float(d.max()), bound, int(np.argmax(d)))
    assert np.all(hits["reserved"] == 0)


def compare_with_order(hits, r_or, m_or, k, n, m):
    """hits equal the oracle's (ranks, mi) list element by element."""
    assert len(hits) == len(r_or)
    np.testing.assert_array_equal(hits["rank"], r_or)
    np.testing.assert_array_equal(hits["mi"], m_or)          # bit-identical FP64
    err = np.abs(hits["mi32"].astype(np.float64) - m_or)
    assert np.all(err <= TOL_REL * np.abs(m_or) + TOL_ABS), err.max()
    check_est(hits, k, m, m_or)
    if len(hits) <= 5000:
        for h in hits:
            assert tuple(h["snp"][:k]) == oracle.unrank(n, k, int(h["rank"]))
            assert np.all(h["snp"][k:] == 0xFFFFFFFF)
    else:
        for i in np.linspace(0, len(hits) - 1, 2000).astype(int):
            assert tuple(hits[i]["snp"][:k]) == oracle.unrank(n, k, int(hits[i]["rank"]))
        assert np.all(hits["snp"][:, k:] == 0xFFFFFFFF)


def check_hits_against_oracle(G, y, k, top_n, hits, nthreads=0):
    """Full oracle scan and element-by-element comparison."""
    r_or, m_or = oracle.scan(G, y, k, top_n, nthreads=nthreads)
    compare_with_order(hits, r_or, m_or, k, G.shape[0], G.shape[1])


def random_dataset(seed, n, m, frac, mono=0, dup=0):
    rng = np.random.default_rng(seed)
    G = rng.binomial(2, rng.uniform(0.05, 0.5, size=(n, 1)), size=(n, m)).astype(np.uint8)
    y = (rng.random(m) < frac).astype(np.uint8)
    if y.sum() == 0 and frac > 0:
        y[0] = 1
    for i in range(mono):
        G[i] = 1
    for i in range(dup):
        G[n - 1 - i] = G[i + mono]
    return G, y


# ---------------------------------------------------------------------------
# order-2 workload (100 variants x 1600 samples): every table, and the result
# ---------------------------------------------------------------------------

def test_order2_small_all_tables():
    d = synth.order2_small()
    say("case: order2 100x1600 all tables")
    total = math.comb(d.n, 2)
    ranks = np.arange(total, dtype=np.uint64)
    gpu = fiuncho.contingency(d.genotypes, d.phenotype, 2, ranks)
    _, ref = oracle.score_ranks(d.genotypes, d.phenotype, 2, ranks, want_tables=True)
    np.testing.assert_array_equal(gpu, ref)


def test_order2_small_scan():
    d = synth.order2_small()
    say("case: order2 100x1600 scan top-10")
    hits = fiuncho.scan(d.genotypes, d.phenotype, 2, d.top_n)
    check_hits_against_oracle(d.genotypes, d.phenotype, 2, d.top_n, hits)
    assert tuple(hits[0]["snp"][:2]) == d.planted[0]


# ---------------------------------------------------------------------------
# small ragged cases, every order, full oracle comparison
# ---------------------------------------------------------------------------

CASES = [
    # seed, n, m, case fraction, order, top_n, monomorphic, duplicated
    (1, 30, 130, 0.5, 1, 5, 0, 0),
    (2, 40, 64, 0.5, 2, 7, 0, 0),
    (3, 70, 200, 0.3, 2, 50, 2, 3),
    (4, 31, 1, 1.0, 2, 3, 0, 0),           # a single sample (one empty class)
    (5, 45, 257, 0.7, 3, 20, 1, 2),
    (6, 25, 65, 0.02, 3, 40, 0, 0),        # one or two cases only
    (7, 18, 300, 0.5, 4, 15, 0, 1),
    (8, 14, 190, 0.4, 5, 10, 1, 1),
    (9, 10, 77, 0.5, 6, 9, 0, 0),
    (10, 9, 50, 0.5, 8, 5, 0, 0),
    (11, 12, 129, 0.5, 3, 300, 0, 0),      # top_n > C(n, k)
    (12, 5, 99, 0.5, 5, 4, 0, 0),          # n == k: a single combination
    (13, 130, 70, 0.5, 2, 2048, 0, 0),     # top_n beyond one LDS sort of results
    (14, 30, 200, 0.5, 6, 20, 1, 1),       # orders 6-8 at 20-30 variants
    (15, 24, 150, 0.45, 7, 20, 0, 1),
    (16, 22, 97, 0.5, 8, 15, 1, 0),
    (17, 13, 88, 0.5, 7, 1716, 0, 0),      # every combination of order 7
    (18, 48, 200, 0.5, 6, 30, 1, 1),       # order 6 at 48 variants (1.2e7 combinations)
]


# counting kernels of the small cases: the rule's choice, the popcount kernel
# (orders 2 and 3 forced off the matrix cores and the pair tables), the
# order-3 pair-table kernel
KERNEL_ENV = {"auto": {}, "popcount": {"FIUNCHO_ORDER2_MFMA": "0", "FIUNCHO_ORDER3_PAIRS": "0"},
              "pairs": {"FIUNCHO_ORDER3_PAIRS": "1"}}


@pytest.mark.parametrize("kernel", list(KERNEL_ENV))
@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}-n{c[1]}-m{c[2]}-k{c[4]}" for c in CASES])
def test_small_cases(case, kernel, monkeypatch):
    seed, n, m, frac, k, top, mono, dup = case
    if kernel == "pairs" and k != 3:
        pytest.skip("the pair-table kernel serves order 3 only")
    for name, val in KERNEL_ENV[kernel].items():
        monkeypatch.setenv(name, val)
    say(f"case: {case} kernel={kernel}")
    G, y = random_dataset(seed, n, m, frac, mono, dup)
    hits = fiuncho.scan(G, y, k, top)
    check_hits_against_oracle(G, y, k, top, hits)
    # tables of every hit
    if len(hits):
        gpu = fiuncho.contingency(G, y, k, hits["rank"])
        _, ref = oracle.score_ranks(G, y, k, hits["rank"], want_tables=True)
        np.testing.assert_array_equal(gpu, ref)


def test_empty_class_returns_first_ranks():
    say("case: empty class")
    G, _ = random_dataset(20, 12, 90, 0.5)
    y = np.zeros(90, np.uint8)
    hits = fiuncho.scan(G, y, 3, 25)
    np.testing.assert_array_equal(hits["rank"], np.arange(25))
    assert np.all(hits["mi"] == 0.0)
    check_hits_against_oracle(G, y, 3, 25, hits)


def test_all_monomorphic_ties_go_to_lowest_ranks():
    say("case: monomorphic ties")
    G = np.ones((20, 150), np.uint8)
    y = (np.arange(150) % 3 == 0).astype(np.uint8)
    hits = fiuncho.scan(G, y, 2, 30)
    np.testing.assert_array_equal(hits["rank"], np.arange(30))
    check_hits_against_oracle(G, y, 2, 30, hits)


def test_duplication_gives_zero_mi():
    """Every sample once as a control and once as a case: MI = 0 exactly in
    real arithmetic for every combination."""
    say("case: duplication")
    G, _ = random_dataset(21, 16, 120, 0.5)
    G2 = np.concatenate([G, G], axis=1)
    y2 = np.array([0] * 120 + [1] * 120, np.uint8)
    hits = fiuncho.scan(G2, y2, 3, 20)
    assert np.all(np.abs(hits["mi"]) <= 1e-14)
    assert np.all(np.abs(hits["mi32"]) <= 1e-9)
    check_hits_against_oracle(G2, y2, 3, 20, hits)


def test_deterministic():
    G, y = random_dataset(22, 60, 333, 0.4, 0, 4)
    a = fiuncho.scan(G, y, 3, 64)
    b = fiuncho.scan(G, y, 3, 64)
    assert a.tobytes() == b.tobytes()


# ---------------------------------------------------------------------------
# full-size workloads: the complete oracle scan
# ---------------------------------------------------------------------------

_FULL = {}


def full_oracle(d):
    """Oracle result of a named workload, computed once per test session on
    every host CPU."""
    key = (d.name, d.order, d.top_n)
    if key not in _FULL:
        say(f"case: {d.name} oracle scan on {oracle.host_threads()} host threads")
        _FULL[key] = oracle.scan(d.genotypes, d.phenotype, d.order, d.top_n)
    return _FULL[key]


def sampled_condition(d, hits, n_sample, seed):
    """Necessary condition of the top-N set on sampled ranks the oracle scores
    one by one: none of them beats the last hit unless it is a hit, and their
    tables equal the library's."""
    k, G, y = d.order, d.genotypes, d.phenotype
    total = math.comb(d.n, k)
    rng = np.random.default_rng(seed)
    ranks = np.unique(rng.integers(0, total, size=n_sample, dtype=np.uint64))
    say(f"case: {d.name} sampled {len(ranks)} ranks")
    mi_s = oracle.score_ranks(G, y, k, ranks)
    last_mi, last_rank = hits[-1]["mi"], hits[-1]["rank"]
    in_hits = np.isin(ranks, hits["rank"])
    beats = (mi_s > last_mi) | ((mi_s == last_mi) & (ranks < last_rank))
    assert not np.any(beats & ~in_hits)
    sub = ranks[:2000]
    _, tab_s = oracle.score_ranks(G, y, k, sub, want_tables=True)
    np.testing.assert_array_equal(fiuncho.contingency(G, y, k, sub), tab_s)


def full_size_check(d, n_sample, seed, full=True):
    """The whole search of a workload against the oracle: with ``full`` the
    complete oracle scan (rank for rank, FP64 bit for bit); else the hits'
    exact values and a sampled necessary condition."""
    k = d.order
    G, y = d.genotypes, d.phenotype
    say(f"case: {d.name} full scan")
    hits = fiuncho.scan(G, y, k, d.top_n)
    assert len(hits) == d.top_n
    mi_or, tab_or = oracle.score_ranks(G, y, k, hits["rank"], want_tables=True)
    np.testing.assert_array_equal(hits["mi"], mi_or)
    np.testing.assert_array_equal(fiuncho.contingency(G, y, k, hits["rank"]), tab_or)
    order = np.lexsort((hits["rank"], -hits["mi"]))
    np.testing.assert_array_equal(order, np.arange(len(hits)))
    check_est(hits, k, d.m, mi_or)
    # the planted interaction of this order ranks first
    planted = [p for p in d.planted if len(p) == k]
    if planted:
        assert tuple(hits[0]["snp"][:k]) == planted[0]
    if full:
        r_or, m_or = full_oracle(d)
        compare_with_order(hits, r_or, m_or, k, d.n, d.m)
    if n_sample:
        sampled_condition(d, hits, n_sample, seed)
    return hits


def test_order3_main_workload():
    full_size_check(synth.order3_main(), 2000, 31)


def test_order3_main_workload_pair_kernel(monkeypatch):
    monkeypatch.setenv("FIUNCHO_ORDER3_PAIRS", "1")
    full_size_check(synth.order3_main(), 2000, 34)


def test_order2_dense_workload():
    full_size_check(synth.order2_dense(), 2000, 32)


def test_order2_dense_workload_popcount_kernel(monkeypatch):
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "0")
    full_size_check(synth.order2_dense(), 2000, 33)


def test_order4_high_order_workload():
    full_size_check(synth.high_order(4), 2000, 34)


def test_order4_high_order_workload_popcount_kernel(monkeypatch):
    monkeypatch.setenv("FIUNCHO_ORDER4_TRIPLES", "0")
    full_size_check(synth.high_order(4), 2000, 35)


@pytest.mark.parametrize("triples", ["0", "1"])
def test_order4_both_kernels(triples, monkeypatch):
    """Order 4 through the generic kernel and through the inclusion-exclusion
    kernel with triple tables, on ragged sizes around the 64-variant and
    64-sample block edges."""
    monkeypatch.setenv("FIUNCHO_ORDER4_TRIPLES", triples)
    for seed, n, m, frac in ((50, 4, 90, 0.5), (51, 9, 64, 0.3), (52, 33, 129, 0.5),
                             (53, 66, 200, 0.45), (54, 70, 65, 0.6)):
        say(f"case: order4 triples={triples} seed={seed} n={n} m={m}")
        G, y = random_dataset(seed, n, m, frac, 1 if n > 5 else 0, 1 if n > 5 else 0)
        top = min(37, math.comb(n, 4))
        hits = fiuncho.scan(G, y, 4, top)
        check_hits_against_oracle(G, y, 4, top, hits)


# ---------------------------------------------------------------------------
# batched form on device pointers
# ---------------------------------------------------------------------------

def test_batch_matches_oracle_per_job():
    import torch

    jobs = synth.batch_jobs(12, scale=0.04)
    say("case: batch of", len(jobs), [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    res = b.results()
    for d, (status, hits) in zip(jobs, res):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)
    # a second run on the same workspace gives the same bytes
    b.run()
    res2 = b.results()
    for (s1, h1), (s2, h2) in zip(res, res2):
        assert s1 == s2 and h1.tobytes() == h2.tobytes()
    torch.cuda.synchronize()


def test_batch_device_validation():
    import torch

    d = synth.generate(20, 100, seed=5, order=2, top_n=5)
    bad = synth.generate(20, 100, seed=6, order=2, top_n=5)
    bad.genotypes[3, 17] = 7
    b = fiuncho.DeviceBatch([d, bad])
    b.run()
    res = b.results()
    assert res[0][0] == 0 and len(res[0][1]) == 5
    assert res[1][0] == fiuncho.E_GENOTYPE and len(res[1][1]) == 0
    torch.cuda.synchronize()


def test_batch_graph_replay():
    """The batched call captured in a HIP graph and replayed several times,
    with eager work and synchronisations in between: every replay equals the
    eager result (and the oracle)."""
    import torch

    jobs = synth.batch_jobs(6, scale=0.05)
    say("case: graph replay", [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    eager = b.results()
    for d, (status, hits) in zip(jobs, eager):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)
    b.capture()
    for rep in range(3):
        for o in b.out:
            o.zero_()
        b.n_out.zero_()
        b.status.fill_(99)
        torch.cuda.synchronize()
        b.replay()
        got = b.results()
        for (s1, h1), (s2, h2) in zip(eager, got):
            assert s1 == s2 and h1.tobytes() == h2.tobytes(), rep
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()


@pytest.mark.parametrize("pairs", ["0", "1"])
def test_order3_both_paths(pairs, monkeypatch):
    """Order 3 through the generic popcount kernel (FIUNCHO_ORDER3_PAIRS=0)
    and through the inclusion-exclusion kernel with pair tables (1)."""
    monkeypatch.setenv("FIUNCHO_ORDER3_PAIRS", pairs)
    for seed, n, m, frac in ((40, 67, 321, 0.45), (41, 130, 128, 0.5), (42, 9, 700, 0.2)):
        say(f"case: order3 pairs={pairs} seed={seed} n={n} m={m}")
        G, y = random_dataset(seed, n, m, frac, 1, 2)
        hits = fiuncho.scan(G, y, 3, 37)
        check_hits_against_oracle(G, y, 3, 37, hits)


# ---------------------------------------------------------------------------
# precision of the single-precision scores
# ---------------------------------------------------------------------------

def fp32_bound(k, m):
    u = 2.0 ** -24
    return 2 * u * (6 * math.log(m) + (3 ** k + 4) * math.log(2))


def test_scores_of_every_order2_pair():
    d = synth.order2_small()
    ranks = np.arange(math.comb(d.n, 2), dtype=np.uint64)
    est, m32, m64 = fiuncho.score(d.genotypes, d.phenotype, 2, ranks)
    ref = oracle.score_ranks(d.genotypes, d.phenotype, 2, ranks)
    np.testing.assert_array_equal(m64, ref)
    assert np.all(np.abs(m32 - ref) <= TOL_REL * np.abs(ref) + TOL_ABS)
    assert np.all(np.abs(est - ref) <= fp32_bound(2, d.m))


@pytest.mark.parametrize("order,count", [(4, 1_000_000), (5, 200_000)])
def test_precision_sample_high_order(order, count):
    """FP32-vs-FP64 error on a seeded sample of combinations of the
    200-variant x 4,000-sample high-order workload."""
    d = synth.high_order(order)
    total = math.comb(d.n, order)
    rng = np.random.default_rng(55)
    ranks = np.unique(rng.integers(0, total, size=count, dtype=np.uint64))
    say(f"case: precision order {order}, {len(ranks)} combinations")
    est, m32, m64 = fiuncho.score(d.genotypes, d.phenotype, order, ranks)
    sub = ranks[:20000]
    np.testing.assert_array_equal(m64[:20000], oracle.score_ranks(d.genotypes, d.phenotype, order, sub))
    rel = np.abs(m32.astype(np.float64) - m64) / np.maximum(np.abs(m64), 1e-300)
    absd = np.abs(m32.astype(np.float64) - m64)
    say(f"order {order}: mi32 rel err max {rel.max():.3e} median {np.median(rel):.3e}, "
        f"abs max {absd.max():.3e}; est abs err max {np.abs(est - m64).max():.3e} "
        f"(bound {fp32_bound(order, d.m):.3e})")
    assert np.all(absd <= TOL_REL * np.abs(m64) + TOL_ABS)
    assert np.all(np.abs(est - m64) <= fp32_bound(order, d.m))


# ---------------------------------------------------------------------------
# shards: one GPU's share of a search split across several
# ---------------------------------------------------------------------------

def _merge(hit_lists, top_n):
    allh = np.concatenate(hit_lists)
    order = np.lexsort((allh["rank"], -allh["mi"]))
    return allh[order][:top_n]


def _run_shards(G, y, k, top_n, P):
    d = synth.Dataset(G, y, k, top_n)
    b = fiuncho.DeviceBatch([d] * P, shards=[(s, P) for s in range(P)])
    b.run()
    res = b.results()
    for status, _ in res:
        assert status == 0
    return [h for _, h in res]


@pytest.mark.parametrize("case", [(700, 300, 1, 20, 3), (300, 500, 2, 50, 7), (150, 400, 3, 40, 5),
                                  (60, 300, 4, 30, 4), (30, 200, 5, 10, 3)])
def test_shards_merge_to_full_result(case):
    """The top-N lists of all shards, merged under the total order, equal the
    full search (the oracle's)."""
    n, m, k, top_n, P = case
    say("case: shards", case)
    G, y = random_dataset(100 + k, n, m, 0.5)
    lists = _run_shards(G, y, k, top_n, P)
    ranks = np.concatenate([h["rank"] for h in lists])
    assert len(np.unique(ranks)) == len(ranks)
    check_hits_against_oracle(G, y, k, top_n, _merge(lists, top_n))


@pytest.mark.parametrize("n,k,P", [(1500, 1, 3), (60, 2, 7), (5, 2, 3), (20, 3, 4), (14, 4, 5),
                                   (11, 5, 3)])
def test_shards_cover_every_combination_once(n, k, P):
    """With top_n at least C(n, k) each shard returns its whole share: its
    size is the host's tile count for that shard, the shares are disjoint and
    cover every rank, and every score is the oracle's."""
    say("case: shard cover", n, k, P)
    G, y = random_dataset(7, n, 150, 0.4)
    total = math.comb(n, k)
    lists = _run_shards(G, y, k, total, P)
    sizes = fiuncho.shard_counts(n, 150, k, P, fiuncho.TILE_ROUND_ROBIN)
    assert [len(h) for h in lists] == sizes.tolist()
    ranks = np.sort(np.concatenate([h["rank"] for h in lists]))
    np.testing.assert_array_equal(ranks, np.arange(total, dtype=np.uint64))
    for h in lists:
        if len(h):
            np.testing.assert_array_equal(h["mi"], oracle.score_ranks(G, y, k, h["rank"]))


def test_shards_with_an_empty_class():
    n, k, top_n, P = 40, 3, 50, 4
    G, y = random_dataset(9, n, 100, 0.0)
    assert y.sum() == 0
    lists = _run_shards(G, y, k, top_n, P)
    total = math.comb(n, k)
    for s, h in enumerate(lists):
        want = min(top_n, (total - s + P - 1) // P)
        np.testing.assert_array_equal(h["rank"], s + P * np.arange(want, dtype=np.uint64))
        assert np.all(h["mi"] == 0.0)
    np.testing.assert_array_equal(_merge(lists, top_n)["rank"], np.arange(top_n, dtype=np.uint64))


# ---------------------------------------------------------------------------
# kernel choice: autotuning and the plan upload flag
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,k", [(300, 500, 2), (70, 300, 3)])
def test_autotune_then_search(n, m, k):
    say(f"case: autotune n={n} m={m} k={k}")
    try:
        kern = fiuncho.autotune(n, m, k, reps=2)
        assert kern in ((fiuncho.KERNEL_POPCOUNT, fiuncho.KERNEL_MFMA, fiuncho.KERNEL_MFMA_FP4) if k == 2 else
                        (fiuncho.KERNEL_POPCOUNT, fiuncho.KERNEL_PAIRS, fiuncho.KERNEL_MFMA,
                         fiuncho.KERNEL_MFMA_FP4))
        assert fiuncho.get_kernel(n, m, k) == kern
        kk, wps = fiuncho.get_config(n, m, k)
        say(f"autotuned: kernel {kk}, waves per SIMD {wps}")
        assert kk == kern and wps in (0, 1, 2)
        G, y = random_dataset(60 + k, n, m, 0.5)
        fiuncho.set_profiling(True)
        b = fiuncho.DeviceBatch([synth.Dataset(G, y, k, 30)])
        b.run()
        (status, hits), = b.results()
        prof = fiuncho.get_profile()
        fiuncho.set_profiling(False)
        assert status == 0
        assert prof["kernels"] == 1 << kern
        check_hits_against_oracle(G, y, k, 30, hits)
    finally:
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_AUTO)


def test_plan_upload_flag_after_workspace_reuse():
    """A workspace overwritten between calls: with FIUNCHO_UPLOAD_PLAN the
    next call uploads the plan again and the results are right."""
    d = synth.generate(80, 400, seed=12, order=3, top_n=20)
    b = fiuncho.DeviceBatch([d])
    b.run()
    first = b.results()
    b.ws.fill_(0)
    b.run(upload_plan=True)
    again = b.results()
    assert first[0][0] == 0 and first[0][1].tobytes() == again[0][1].tobytes()
    check_hits_against_oracle(d.genotypes, d.phenotype, 3, 20, again[0][1])


# ---------------------------------------------------------------------------
# size extremes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mfma", ["0", "1", "4"])
def test_maximum_samples(mfma, monkeypatch):
    """samples = 2^24 - 1, the largest accepted: counts far above 2^16, the
    widest single-precision bound, 262,146-word rows."""
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", mfma)
    n, m = 5, (1 << 24) - 1
    rng = np.random.default_rng(70)
    G = rng.integers(0, 3, (n, m), dtype=np.uint8)
    y = (rng.random(m) < 0.45).astype(np.uint8)
    for k in ((2,) if mfma != "0" else (1, 2, 3)):
        say(f"case: maximum samples k={k} mfma={mfma}")
        hits = fiuncho.scan(G, y, k, 5)
        check_hits_against_oracle(G, y, k, 5, hits)


def test_many_variants_order2():
    """30,000 variants (4.5e8 pairs, matrix-core kernel by the rule)."""
    full_size_check(synth.generate(30000, 128, seed=71, order=2, top_n=50, name="order2-30000x128"),
                    20000, 72)


def test_many_variants_order3():
    """3,000 variants (4.5e9 triples, 295 MB of pair tables): the hits'
    exact values and a sampled condition (a full oracle scan would take
    minutes)."""
    full_size_check(synth.generate(3000, 64, seed=73, order=3, top_n=50, name="order3-3000x64"),
                    200000, 74, full=False)


# ---------------------------------------------------------------------------
# exact ties at the cut-off, beyond one LDS sort of kept candidates
# ---------------------------------------------------------------------------

def _tie_dataset(seed, kind, n_tied=200, n_other=20, m=300):
    """n_tied variants that are all identical (one class-associated genotype
    row copied) or all monomorphic, then n_other random variants."""
    rng = np.random.default_rng(seed)
    y = (rng.random(m) < 0.5).astype(np.uint8)
    other = rng.binomial(2, rng.uniform(0.05, 0.5, size=(n_other, 1)), size=(n_other, m)).astype(np.uint8)
    if kind == "identical":
        row = np.where(rng.random(m) < 0.7, y * 2, rng.integers(0, 3, m)).astype(np.uint8)
        tied = np.repeat(row[None, :], n_tied, axis=0)
    else:
        tied = np.ones((n_tied, m), np.uint8)
    return np.concatenate([tied, other]), y


# (kind, other variants, top_n): 200 identical variants alone give C(200, 2) =
# 19,900 pairs with one table, all tied at the top (top_n 10: the kept
# candidates are reduced to the results by radix selection; 9,000: the
# results are ordered by the multi-block sort); with 20 random variants each
# of them pairs with the 200 identical ones in 200-way ties; monomorphic
# variants pair with each other at MI 0 (19,900 ties, reached by top_n 5,000)
# and with each random variant at that variant's MI (200-way ties)
TIES = [("identical", 0, 10), ("identical", 0, 9000), ("identical", 20, 10), ("monomorphic", 20, 500),
        ("monomorphic", 20, 5000)]


@pytest.mark.parametrize("kind,n_other,top_n", TIES)
def test_ties_at_the_cut_off(kind, n_other, top_n):
    """Exact ties at the cut-off, up to far more than one LDS sort of kept
    candidates holds: the result is the unique top_n under (MI descending,
    rank ascending), as the oracle's."""
    G, y = _tie_dataset(90, kind, n_other=n_other)
    say(f"case: ties {kind} +{n_other} top_n={top_n}")
    hits = fiuncho.scan(G, y, 2, top_n)
    check_hits_against_oracle(G, y, 2, top_n, hits)
    if n_other == 0:
        np.testing.assert_array_equal(hits["rank"], np.arange(top_n))


# ---------------------------------------------------------------------------
# the order-5 high-order workload, every combination (2.5e9)
# ---------------------------------------------------------------------------

def test_order5_full_workload():
    """The whole order-5 search of the 200-variant x 4,000-sample workload:
    the planted 5-set first, the hits' tables and FP64 scores equal the
    oracle's, every estimate within its bound, the order total, and no
    sampled combination (2e6 scored by the oracle) beats the last hit."""
    d = synth.high_order(5)
    full_size_check(d, 2_000_000, 58, full=False)


# ---------------------------------------------------------------------------
# the batch of 64 uneven datasets at full size
# ---------------------------------------------------------------------------

def test_batch64_full_size():
    """All 64 uneven jobs of the batched workload in one call (device
    pointers): every job's hits have the oracle's tables, FP64 scores and
    order, estimates within their bounds and the planted set first; jobs the
    oracle scans in about a second (C(n, k) m <= 4e10: the 32 order-2 jobs and
    two order-3 jobs) are compared with the complete oracle scan, the others
    on 20,000 sampled ranks."""
    jobs = synth.batch_jobs(64)
    say("case: batch64 full size")
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    res = b.results()
    full = 0
    for d, (status, hits) in zip(jobs, res):
        assert status == 0, d.name
        k = d.order
        assert len(hits) == d.top_n
        mi_or = oracle.score_ranks(d.genotypes, d.phenotype, k, hits["rank"])
        np.testing.assert_array_equal(hits["mi"], mi_or)
        check_est(hits, k, d.m, mi_or)
        np.testing.assert_array_equal(np.lexsort((hits["rank"], -hits["mi"])), np.arange(len(hits)))
        assert tuple(hits[0]["snp"][:k]) == d.planted[0], d.name
        if math.comb(d.n, k) * d.m <= 4e10:
            r_or, m_or = oracle.scan(d.genotypes, d.phenotype, k, d.top_n)
            compare_with_order(hits, r_or, m_or, k, d.n, d.m)
            full += 1
        else:
            sampled_condition(d, hits, 20000, 900 + int(d.name[5:].split("-")[0]))
    say(f"batch64: {full} jobs against the complete oracle scan")
    assert full >= 32


# ---------------------------------------------------------------------------
# a workspace in memory that held an earlier batch's workspace
# ---------------------------------------------------------------------------

def test_new_batch_in_reused_memory():
    """A batch whose workspace reuses freed memory of an earlier batch of the
    same shapes (the caching allocator hands the block back), overwritten in
    between: the new batch's first run uploads its plan, so its results are
    the oracle's."""
    import torch

    d = synth.generate(90, 500, seed=14, order=3, top_n=25)
    a = fiuncho.DeviceBatch([d])
    a.run()
    first = a.results()
    ptr = a.ws.data_ptr()
    nbytes = a.ws.numel()
    del a
    junk = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    reused = junk.data_ptr() == ptr
    del junk
    b = fiuncho.DeviceBatch([d])
    say(f"case: reused workspace memory (same block: {reused and b.ws.data_ptr() == ptr})")
    b.run()
    (status, hits), = b.results()
    assert status == 0
    assert hits.tobytes() == first[0][1].tobytes()
    check_hits_against_oracle(d.genotypes, d.phenotype, 3, 25, hits)


@pytest.mark.parametrize("wps", [1, 2])
def test_waves_per_simd_limit(wps):
    """A configuration that limits the counting launch to 1 or 2 waves per
    SIMD gives the same result as full occupancy (a persistent grid of fewer
    workgroups draws every tile)."""
    G, y = random_dataset(64 + wps, 150, 700, 0.45, 1, 1)
    try:
        fiuncho.set_config(150, 700, 3, fiuncho.KERNEL_MFMA_FP4, wps)
        assert fiuncho.get_config(150, 700, 3) == (fiuncho.KERNEL_MFMA_FP4, wps)
        hits = fiuncho.scan(G, y, 3, 40)
    finally:
        fiuncho.set_config(150, 700, 3, fiuncho.KERNEL_AUTO, 0)
    check_hits_against_oracle(G, y, 3, 40, hits)
