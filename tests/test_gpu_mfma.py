"""GPU parity of the matrix-core paths (order 2: FIUNCHO_ORDER2_MFMA, order
3: FIUNCHO_ORDER3_MFMA; 1 = int8 operands, 4 = FP4 operands): the one-hot
contraction must give the same tables, top-N set and FP64 scores as the
oracle, like the popcount path, in either operand format."""
import math

import numpy as np
import pytest

import oracle
from paper_2201_03331_amd import fiuncho, synth
from test_gpu_parity import check_hits_against_oracle, full_size_check, random_dataset, say, _merge, _run_shards

pytestmark = pytest.mark.gpu


# operand formats of the matrix-core kernels: environment value, test id
FORMATS = dict(params=["1", "4"], ids=["int8", "fp4"])


@pytest.fixture(**FORMATS)
def mfma(monkeypatch, request):
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", request.param)
    return request.param


# n around the 16/32/64-variant block edges, m around the 32/64-sample steps
CASES = [(2, 50, 0.5), (3, 64, 0.5), (17, 31, 0.4), (33, 100, 0.3), (64, 640, 0.5),
         (65, 129, 0.7), (96, 65, 0.5), (130, 1000, 0.5), (257, 77, 0.45)]


@pytest.mark.parametrize("n,m,frac", CASES)
def test_order2_mfma_small(n, m, frac, mfma):
    say(f"case: mfma order 2 n={n} m={m}")
    G, y = random_dataset(31 + n, n, m, frac, 1 if n > 4 else 0, 1 if n > 4 else 0)
    top = min(40, math.comb(n, 2))
    hits = fiuncho.scan(G, y, 2, top)
    check_hits_against_oracle(G, y, 2, top, hits)


def test_order2_mfma_every_pair(mfma):
    """top_n >= C(n, 2): every pair is returned, with the oracle's score."""
    n = 60
    G, y = random_dataset(77, n, 300, 0.5)
    hits = fiuncho.scan(G, y, 2, math.comb(n, 2) + 5)
    assert len(hits) == math.comb(n, 2)
    np.testing.assert_array_equal(np.sort(hits["rank"]), np.arange(math.comb(n, 2), dtype=np.uint64))
    np.testing.assert_array_equal(hits["mi"], oracle.score_ranks(G, y, 2, hits["rank"]))
    check_hits_against_oracle(G, y, 2, len(hits), hits)


def test_order2_mfma_workloads(mfma):
    d = synth.order2_small()
    check_hits_against_oracle(d.genotypes, d.phenotype, 2, d.top_n,
                              fiuncho.scan(d.genotypes, d.phenotype, 2, d.top_n))
    full_size_check(synth.order2_dense(), 2000, 52)


def test_order2_mfma_in_a_mixed_batch(mfma):
    """Order-2 jobs on the matrix cores and order-3 jobs on the popcount
    kernel in one batched call."""
    jobs = synth.batch_jobs(10, scale=0.04)
    say("case: mixed batch", [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    for d, (status, hits) in zip(jobs, b.results()):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)


@pytest.mark.parametrize("n,P", [(300, 7), (60, 3), (5, 3)])
def test_order2_mfma_shards(n, P, mfma):
    G, y = random_dataset(88 + n, n, 200, 0.5)
    top = min(50, math.comb(n, 2))
    lists = _run_shards(G, y, 2, top, P)
    check_hits_against_oracle(G, y, 2, top, _merge(lists, top))
    if math.comb(n, 2) <= 50000:
        full = _run_shards(G, y, 2, math.comb(n, 2), P)
        sizes = fiuncho.shard_counts(n, 200, 2, P, fiuncho.TILE_ROUND_ROBIN)
        assert [len(h) for h in full] == sizes.tolist()


# ---------------------------------------------------------------------------
# order 3: prefix pairs x last variants on the matrix cores
# ---------------------------------------------------------------------------

@pytest.fixture(**FORMATS)
def mfma3(monkeypatch, request):
    monkeypatch.setenv("FIUNCHO_ORDER3_MFMA", request.param)
    return request.param


# n around the 8-prefix fragments, 32-prefix groups and 64-variant blocks
CASES3 = [(3, 50, 0.5), (9, 64, 0.4), (17, 31, 0.5), (34, 129, 0.3), (66, 200, 0.5), (100, 65, 0.6)]


@pytest.mark.parametrize("n,m,frac", CASES3)
def test_order3_mfma_small(n, m, frac, mfma3):
    say(f"case: mfma order 3 n={n} m={m}")
    G, y = random_dataset(131 + n, n, m, frac, 1 if n > 5 else 0, 1 if n > 5 else 0)
    top = min(40, math.comb(n, 3))
    hits = fiuncho.scan(G, y, 3, top)
    check_hits_against_oracle(G, y, 3, top, hits)


def test_order3_mfma_every_triple(mfma3):
    n = 23  # every combination is returned
    G, y = random_dataset(177, n, 150, 0.5)
    hits = fiuncho.scan(G, y, 3, math.comb(n, 3))
    assert len(hits) == math.comb(n, 3)
    np.testing.assert_array_equal(np.sort(hits["rank"]), np.arange(math.comb(n, 3), dtype=np.uint64))
    check_hits_against_oracle(G, y, 3, len(hits), hits)


def test_order3_mfma_workload(mfma3):
    full_size_check(synth.order3_main(), 2000, 53)


def test_order3_mfma_shards_and_batch(mfma3, monkeypatch):
    # order 2 on the matrix cores in the other operand format
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "4" if mfma3 == "1" else "1")
    G, y = random_dataset(93, 120, 180, 0.5)
    lists = _run_shards(G, y, 3, 40, 5)
    check_hits_against_oracle(G, y, 3, 40, _merge(lists, 40))
    # both matrix-core orders and the popcount kernel in one batch
    jobs = synth.batch_jobs(6, scale=0.04) + [synth.generate(30, 300, seed=9, order=4, top_n=5)]
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    for d, (status, hits) in zip(jobs, b.results()):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)


def test_matrix_core_batch_graph_replay(mfma, mfma3):
    """Both matrix-core kernels captured in a HIP graph and replayed, with eager
    work in between: every replay equals the eager result."""
    import torch

    jobs = synth.batch_jobs(6, scale=0.05)
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
        torch.cuda.synchronize()
        b.replay()
        got = b.results()
        for (s1, h1), (s2, h2) in zip(eager, got):
            assert s1 == s2 and h1.tobytes() == h2.tobytes(), rep
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()


def test_both_operand_formats_in_one_batch(monkeypatch):
    """Order-2 and order-3 jobs on the matrix cores, int8 for some shapes and
    FP4 for others, next to popcount jobs, in one batched call: each of the
    four matrix-core groups runs its own launch over its own tiles."""
    for v in ("FIUNCHO_ORDER2_MFMA", "FIUNCHO_ORDER3_MFMA", "FIUNCHO_ORDER3_PAIRS"):
        monkeypatch.delenv(v, raising=False)
    jobs = [synth.generate(150, 300, seed=21, order=2, top_n=20),
            synth.generate(300, 700, seed=22, order=2, top_n=20),
            synth.generate(60, 400, seed=23, order=3, top_n=20),
            synth.generate(130, 200, seed=24, order=3, top_n=20),
            synth.generate(40, 500, seed=25, order=3, top_n=10),
            synth.generate(70, 900, seed=26, order=2, top_n=10)]
    kinds = [fiuncho.KERNEL_MFMA, fiuncho.KERNEL_MFMA_FP4, fiuncho.KERNEL_MFMA_FP4, fiuncho.KERNEL_MFMA,
             fiuncho.KERNEL_PAIRS, fiuncho.KERNEL_POPCOUNT]
    try:
        for d, kind in zip(jobs, kinds):
            fiuncho.set_kernel(d.n, d.m, d.order, kind)
        for d, kind in zip(jobs, kinds):
            assert fiuncho.get_kernel(d.n, d.m, d.order) == kind
        fiuncho.set_profiling(True)
        b = fiuncho.DeviceBatch(jobs)
        b.run()
        res = b.results()
        prof = fiuncho.get_profile()
        fiuncho.set_profiling(False)
        assert prof["kernels"] == sum(1 << k for k in set(kinds))
        for d, (status, hits) in zip(jobs, res):
            assert status == 0
            check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)
    finally:
        for d in jobs:
            fiuncho.set_kernel(d.n, d.m, d.order, fiuncho.KERNEL_AUTO)


def test_fp4_narrow_and_wide_launches(monkeypatch):
    """FP4 jobs with at most 20,447 samples run the kernel variant that keeps
    counts in 16 bits (f table in LDS); larger ones the 32-bit variant (f
    table in global memory).  Both orders, both variants, one batch."""
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "4")
    monkeypatch.setenv("FIUNCHO_ORDER3_MFMA", "4")
    jobs = [synth.generate(40, 25000, seed=81, order=3, top_n=15),
            synth.generate(70, 3000, seed=82, order=3, top_n=15),
            synth.generate(90, 20447, seed=83, order=2, top_n=15),
            synth.generate(90, 20448, seed=84, order=2, top_n=15)]
    say("case: narrow and wide FP4", [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    for d, (status, hits) in zip(jobs, b.results()):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)


def test_fp4_dual_and_narrow_launches(monkeypatch):
    """Among FP4 jobs with counts in 16 bits, those with at most 8,191 samples
    whose class sizes m0, m1 satisfy bitlen(m0) + bitlen(m1) <= 24 run the
    kernel that accumulates both classes in one FP32 register (class 1 scaled
    by 2^bitlen(m0)); the rest run the two-accumulator kernel over the same
    tiles.  Both score from packed byte offsets (4 x count per class, 16-bit
    halves) when both class sizes are below 16,384.  Jobs at both sides of
    every limit, both orders, one batch."""
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "4")
    monkeypatch.setenv("FIUNCHO_ORDER3_MFMA", "4")
    # (m, cases): 6143 + 2047 and 2047 + 6143 reach 24 bits exactly; 4096 +
    # 4095 needs 25; 8192 samples exceed the dual kernel's table; 16,383
    # controls are the most the packed scoring takes, 16,384 the fewest it
    # leaves to the per-class scoring
    shapes = [(8190, 2047), (8190, 6143), (8191, 4095), (8192, 100), (500, 250),
              (18383, 2000), (18384, 2000)]
    jobs = []
    for order, n in ((2, 70), (3, 30)):
        for i, (m, cases) in enumerate(shapes):
            d = synth.generate(n + i, m, seed=90 + 10 * order + i, order=order, top_n=12,
                               case_fraction=cases / m)
            assert d.m == m and int(d.phenotype.sum()) == cases
            jobs.append(d)
    say("case: dual and narrow FP4", [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    for d, (status, hits) in zip(jobs, b.results()):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)


# ---------------------------------------------------------------------------
# orders 4 and 5: every prefix row on the matrix cores (FP4)
# ---------------------------------------------------------------------------

@pytest.fixture
def rows_kernel():
    """Puts the FP4 matrix-core kernel in the table for the shapes a test
    registers; clears them afterwards."""
    shapes = []

    def use(n, m, k):
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_MFMA_FP4)
        shapes.append((n, m, k))
        assert fiuncho.get_kernel(n, m, k) == fiuncho.KERNEL_MFMA_FP4

    yield use
    for n, m, k in shapes:
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_AUTO)


# n around the 4-prefix groups and 64-variant blocks, m around word edges
CASES45 = [(4, 7, 64, 0.5), (4, 20, 300, 0.4), (4, 35, 130, 0.5), (4, 70, 1000, 0.3),
           (5, 9, 77, 0.5), (5, 14, 190, 0.45), (5, 22, 400, 0.6), (5, 68, 129, 0.5)]


@pytest.mark.parametrize("k,n,m,frac", CASES45)
def test_orders45_rows_small(k, n, m, frac, rows_kernel):
    say(f"case: rows order {k} n={n} m={m}")
    rows_kernel(n, m, k)
    G, y = random_dataset(211 + n + k, n, m, frac, 1 if n > 8 else 0, 1 if n > 8 else 0)
    top = min(30, math.comb(n, k))
    fiuncho.set_profiling(True)
    hits = fiuncho.scan(G, y, k, top)
    prof = fiuncho.get_profile()
    fiuncho.set_profiling(False)
    assert prof["kernels"] == 1 << fiuncho.KERNEL_MFMA_FP4
    check_hits_against_oracle(G, y, k, top, hits)


@pytest.mark.parametrize("k,n", [(4, 15), (5, 13)])
def test_orders45_rows_every_combination(k, n, rows_kernel):
    m = 150
    rows_kernel(n, m, k)
    G, y = random_dataset(300 + k, n, m, 0.5)
    hits = fiuncho.scan(G, y, k, math.comb(n, k))
    assert len(hits) == math.comb(n, k)
    np.testing.assert_array_equal(np.sort(hits["rank"]), np.arange(math.comb(n, k), dtype=np.uint64))
    np.testing.assert_array_equal(hits["mi"], oracle.score_ranks(G, y, k, hits["rank"]))
    check_hits_against_oracle(G, y, k, len(hits), hits)


def test_order4_rows_workload(rows_kernel):
    d = synth.high_order(4)
    rows_kernel(d.n, d.m, 4)
    full_size_check(d, 2000, 57)


def test_orders45_rows_large_samples_fall_back(rows_kernel):
    """More than 20,447 samples: the job runs on the popcount kernel."""
    n, m = 8, 25000
    rows_kernel(n, m, 4)
    G, y = random_dataset(88, n, m, 0.5)
    fiuncho.set_profiling(True)
    hits = fiuncho.scan(G, y, 4, 20)
    prof = fiuncho.get_profile()
    fiuncho.set_profiling(False)
    assert prof["kernels"] == 1 << fiuncho.KERNEL_POPCOUNT
    check_hits_against_oracle(G, y, 4, 20, hits)


def test_orders45_dual_and_two_accumulator_launches(rows_kernel):
    """Orders 4 and 5 on the matrix cores: jobs whose class sizes fit 24 bits
    together, and whose f table fits the dual kernel's LDS (8,192 entries at
    order 4, 20,448 at order 5), run with both classes in one accumulator;
    the rest run the two-accumulator kernel over the same tiles.  Jobs at
    both sides of every limit, both orders, one batch."""
    # (m, cases): 6143 + 2047 reach 24 bits exactly; 4096 + 4095 need 25;
    # 9,000 samples exceed the order-4 dual table; 11,500 + 500 fit 23 bits
    # (dual at order 5 only); 19,447 + 1,000 need 25
    shapes = [(8190, 2047), (8191, 4095), (9000, 4500), (12000, 500), (20447, 1000), (500, 250)]
    jobs = []
    for k, n in ((4, 10), (5, 9)):
        for i, (m, cases) in enumerate(shapes):
            rows_kernel(n + i, m, k)
            d = synth.generate(n + i, m, seed=700 + 10 * k + i, order=k, top_n=12, case_fraction=cases / m)
            assert d.m == m and int(d.phenotype.sum()) == cases
            jobs.append(d)
    say("case: orders 4/5 dual and two-accumulator", [(j.n, j.m, j.order) for j in jobs])
    b = fiuncho.DeviceBatch(jobs)
    b.run()
    for d, (status, hits) in zip(jobs, b.results()):
        assert status == 0
        check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)


def test_every_launch_group_in_one_batch(rows_kernel, monkeypatch):
    """One batch with a job in each matrix-core launch group (orders 2 and 3
    with int8, FP4 and 16-bit-count FP4 operands; orders 4 and 5 with every
    prefix row) and popcount jobs: each group runs over its own tiles."""
    for v in ("FIUNCHO_ORDER2_MFMA", "FIUNCHO_ORDER3_MFMA", "FIUNCHO_ORDER3_PAIRS", "FIUNCHO_ORDER4_TRIPLES"):
        monkeypatch.delenv(v, raising=False)
    specs = [(70, 300, 2, fiuncho.KERNEL_MFMA), (80, 21000, 2, fiuncho.KERNEL_MFMA_FP4),
             (90, 500, 2, fiuncho.KERNEL_MFMA_FP4), (40, 260, 3, fiuncho.KERNEL_MFMA),
             (30, 20500, 3, fiuncho.KERNEL_MFMA_FP4), (50, 700, 3, fiuncho.KERNEL_MFMA_FP4),
             (24, 300, 4, fiuncho.KERNEL_MFMA_FP4), (16, 200, 5, fiuncho.KERNEL_MFMA_FP4),
             (45, 150, 3, fiuncho.KERNEL_PAIRS), (18, 120, 4, fiuncho.KERNEL_TRIPLES),
             (12, 100, 6, fiuncho.KERNEL_POPCOUNT)]
    jobs = []
    try:
        for i, (n, m, k, kind) in enumerate(specs):
            if kind == fiuncho.KERNEL_MFMA_FP4 and k >= 4:
                rows_kernel(n, m, k)
            else:
                fiuncho.set_kernel(n, m, k, kind)
            jobs.append(synth.generate(n, m, seed=500 + i, order=k, top_n=12))
        say("case: every launch group", [(j.n, j.m, j.order) for j in jobs])
        b = fiuncho.DeviceBatch(jobs)
        b.run()
        for d, (status, hits) in zip(jobs, b.results()):
            assert status == 0
            check_hits_against_oracle(d.genotypes, d.phenotype, d.order, d.top_n, hits)
    finally:
        for n, m, k, kind in specs:
            fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_AUTO)
