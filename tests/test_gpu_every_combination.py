"""Every combination through each counting kernel and launch group.

With top_n >= C(n, k) the search keeps and returns every combination, and each
hit carries the plain single-precision MI its counting kernel computed from
its own counts (fiuncho_hit.est).  Comparing those with the oracle's MI of the
same combination, within the rounding bound of that evaluation
(fiuncho_estimate_bound), checks the counting kernel's table of every
combination: one miscounted cell moves MI by about ln(2) / m (about 1e-4 at a
few thousand samples), while the bound is about 1e-6.  The returned list must
also be the oracle's complete ordering (MI descending, rank ascending), rank
for rank and FP64 bit for bit.

Each case forces one kernel for its shape (fiuncho_set_kernel) and checks in
the profile that it ran; the sizes are ragged around the kernels' tile edges
(64 last variants, 32 first variants or prefixes, 16/32/64-sample steps) and
cover both sides of the matrix-core kernels' sample limits (dual: one
accumulator for both classes; narrow: counts in 16 bits; wide: 32 bits).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2201_03331_amd import fiuncho
from test_gpu_parity import compare_with_order, random_dataset, say

pytestmark = pytest.mark.gpu

K = fiuncho
# id, order, n, m, case fraction, kernel
CASES = [
    ("popcount", 1, 300, 333, 0.5, K.KERNEL_POPCOUNT),
    ("popcount", 2, 150, 1000, 0.4, K.KERNEL_POPCOUNT),
    ("popcount", 3, 60, 257, 0.5, K.KERNEL_POPCOUNT),
    ("popcount", 4, 30, 190, 0.45, K.KERNEL_POPCOUNT),
    ("popcount", 5, 22, 130, 0.5, K.KERNEL_POPCOUNT),
    ("popcount", 6, 18, 100, 0.5, K.KERNEL_POPCOUNT),
    ("popcount", 7, 16, 77, 0.6, K.KERNEL_POPCOUNT),
    ("popcount", 8, 14, 65, 0.5, K.KERNEL_POPCOUNT),
    ("pairs", 3, 70, 321, 0.45, K.KERNEL_PAIRS),
    ("triples", 4, 40, 200, 0.5, K.KERNEL_TRIPLES),
    ("int8", 2, 200, 640, 0.5, K.KERNEL_MFMA),
    ("int8", 3, 60, 300, 0.5, K.KERNEL_MFMA),
    # FP4, more than 20,447 samples: 32-bit counts, f table in global memory
    ("fp4-wide", 2, 70, 20500, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-wide", 3, 24, 20600, 0.5, K.KERNEL_MFMA_FP4),
    # FP4, at most 20,447 samples but more than one accumulator can hold for
    # both classes: counts in 16 bits, two accumulators
    ("fp4-narrow", 2, 130, 9000, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-narrow", 3, 40, 9001, 0.5, K.KERNEL_MFMA_FP4),
    # FP4, both classes in one accumulator (bitlen(m0) + bitlen(m1) <= 24)
    ("fp4-dual", 2, 260, 1000, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-dual", 3, 70, 700, 0.5, K.KERNEL_MFMA_FP4),
    # order-3 tiles by block of last variants first: three blocks (jb = 0..2)
    # and a ragged last one
    ("fp4-dual", 3, 150, 200, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-narrow", 3, 135, 9001, 0.5, K.KERNEL_MFMA_FP4),
    # words in pairs: one word per class (the odd step alone), and an even
    # class beside an odd one
    ("fp4-dual", 2, 90, 120, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-dual", 3, 45, 120, 0.5, K.KERNEL_MFMA_FP4),
    ("fp4-dual", 2, 100, 330, 0.4, K.KERNEL_MFMA_FP4),
    ("fp4-dual", 3, 55, 330, 0.4, K.KERNEL_MFMA_FP4),
    # orders 4 and 5, every prefix row on the matrix cores
    ("rows-dual", 4, 30, 400, 0.5, K.KERNEL_MFMA_FP4),
    ("rows-two-acc", 4, 20, 9000, 0.5, K.KERNEL_MFMA_FP4),
    ("rows-dual", 5, 22, 300, 0.5, K.KERNEL_MFMA_FP4),
    ("rows-two-acc", 5, 16, 8200, 0.5, K.KERNEL_MFMA_FP4),
    # order 4, {0,1}^4 cells on the matrix cores and packed triple tables:
    # dual, two accumulators, and one prefix group short of 16 at every row
    ("fp4-triples-dual", 4, 30, 400, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-triples-dual", 4, 37, 1001, 0.3, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-triples-two-acc", 4, 21, 9000, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-triples-two-acc", 4, 18, 16383, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    # order 5, {0,1}^5 cells on the matrix cores and packed quad, triple and
    # pair tables: dual and two accumulators, prefix groups short of 8
    ("fp4-quads-dual", 5, 22, 300, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-quads-dual", 5, 19, 777, 0.35, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-quads-two-acc", 5, 16, 8200, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-quads-two-acc", 5, 13, 16383, 0.45, K.KERNEL_MFMA_FP4_TABLES),
    # the fewest variants: a single combination, and one more variant
    ("fp4-tables-min", 4, 4, 100, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-tables-min", 4, 5, 333, 0.4, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-tables-min", 5, 5, 90, 0.5, K.KERNEL_MFMA_FP4_TABLES),
    ("fp4-tables-min", 5, 6, 257, 0.6, K.KERNEL_MFMA_FP4_TABLES),
]

ENV = ("FIUNCHO_ORDER2_MFMA", "FIUNCHO_ORDER3_MFMA", "FIUNCHO_ORDER3_PAIRS", "FIUNCHO_ORDER4_TRIPLES")


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-k{c[1]}-n{c[2]}-m{c[3]}" for c in CASES])
def test_every_combination(case, monkeypatch):
    name, k, n, m, frac, kernel = case
    for v in ENV:
        monkeypatch.delenv(v, raising=False)
    total = math.comb(n, k)
    G, y = random_dataset(1000 + 10 * k + n, n, m, frac, 1, 1)
    say(f"case: every combination {name} k={k} n={n} m={m} ({total} combinations)")
    try:
        fiuncho.set_kernel(n, m, k, kernel)
        assert fiuncho.get_kernel(n, m, k) == kernel
        fiuncho.set_profiling(True)
        hits = fiuncho.scan(G, y, k, total)
        prof = fiuncho.get_profile()
    finally:
        fiuncho.set_profiling(False)
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_AUTO)
    assert prof["kernels"] == 1 << kernel
    assert len(hits) == total
    r_or, m_or = oracle.order_all(G, y, k)
    compare_with_order(hits, r_or, m_or, k, n, m)
    # the estimates are the kernel's own: not all equal to a recomputation in
    # another summation order, yet every one within the bound
    say(f"{name} k={k}: max |est - mi| = {np.abs(hits['est'] - hits['mi']).max():.3e} "
        f"(bound {fiuncho.estimate_bound(k, m):.3e})")


def test_fp4_triples_large_jobs_use_unpacked_tables(monkeypatch):
    """Order-4 jobs of 16,384 samples or more forced onto the matrix-core
    triple-table kernel run on the popcount triple-table kernel instead (the
    packed tables hold counts below 16,384), with the same results."""
    for v in ENV:
        monkeypatch.delenv(v, raising=False)
    n, m, k = 14, 16384, 4
    G, y = random_dataset(4242, n, m, 0.5, 1, 1)
    try:
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_MFMA_FP4_TABLES)
        fiuncho.set_profiling(True)
        hits = fiuncho.scan(G, y, k, math.comb(n, k))
        prof = fiuncho.get_profile()
    finally:
        fiuncho.set_profiling(False)
        fiuncho.set_kernel(n, m, k, fiuncho.KERNEL_AUTO)
    assert prof["kernels"] == 1 << fiuncho.KERNEL_TRIPLES
    r_or, m_or = oracle.order_all(G, y, k)
    compare_with_order(hits, r_or, m_or, k, n, m)
