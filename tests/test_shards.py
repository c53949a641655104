"""Static work distribution (host-only; no GPU): the paper's (k-1)-prefix
round-robin (section 4.1, Fig. 4; balance metric Eq. 4, section 5.1) and this
library's shard dealing of work tiles, through fiuncho_shard_counts."""
import ctypes
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2201_03331_amd import fiuncho

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_distribution.json")))


def imbalance(counts, n, k):
    """Eq. 4, in percent."""
    p = len(counts)
    mean = math.comb(n, k) / p
    return 100.0 * (float(counts.max()) - mean) / mean


def test_fig4_example():
    f = GOLD["fig4"]
    got = fiuncho.shard_counts(f["variants"], 0, f["order"], f["units"], fiuncho.PREFIX_ROUND_ROBIN)
    assert got.tolist() == f["combinations_per_unit"]


@pytest.mark.parametrize("n,k,p", [(8, 4, 3), (9, 2, 4), (11, 3, 5), (10, 5, 7), (7, 1, 3),
                                   (6, 6, 2), (12, 4, 1), (5, 2, 9)])
def test_prefix_scheme_by_enumeration(n, k, p):
    """Every k-combination goes to the unit of its (k-1)-prefix, whose place is
    its position among the prefixes that have an extension (brute force)."""
    if k == 1:
        want = np.zeros(p, np.uint64)
        want[0] = n
    else:
        prefixes = [c for c in itertools.combinations(range(n), k - 1) if c[-1] < n - 1]
        unit = {c: i % p for i, c in enumerate(prefixes)}
        want = np.zeros(p, np.uint64)
        for c in itertools.combinations(range(n), k):
            want[unit[c[:-1]]] += 1
    got = fiuncho.shard_counts(n, 0, k, p, fiuncho.PREFIX_ROUND_ROBIN)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("scheme", [fiuncho.PREFIX_ROUND_ROBIN, fiuncho.TILE_ROUND_ROBIN])
@pytest.mark.parametrize("n,k", [(1, 1), (300, 1), (2, 2), (130, 2), (3, 3), (70, 3), (200, 3),
                                 (40, 4), (30, 5), (20, 6), (16, 7), (12, 8)])
def test_counts_partition_the_search(scheme, n, k):
    total = math.comb(n, k)
    for p in (1, 2, 3, 7, 64, 1000):
        c = fiuncho.shard_counts(n, 1000, k, p, scheme)
        assert len(c) == p and int(c.sum()) == total, p
    assert fiuncho.shard_counts(n, 1000, k, 1, scheme).tolist() == [total]


@pytest.mark.parametrize("n", [2, 63, 64, 65, 129, 300])
def test_matrix_core_tiles_partition_order2(n, monkeypatch):
    monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "1")
    for p in (1, 3, 8):
        c = fiuncho.shard_counts(n, 1000, 2, p, fiuncho.TILE_ROUND_ROBIN)
        assert int(c.sum()) == math.comb(n, 2)


@pytest.mark.parametrize("n", [3, 4, 66, 67, 130, 131, 300])
def test_matrix_core_tiles_partition_order3(n, monkeypatch):
    """Order-3 matrix-core tiles (rows of (block of last variants, middle
    variant)) hold every triple once: the shards' counts add up to C(n, 3)."""
    monkeypatch.setenv("FIUNCHO_ORDER3_MFMA", "4")
    for p in (1, 3, 8):
        c = fiuncho.shard_counts(n, 1000, 3, p, fiuncho.TILE_ROUND_ROBIN)
        assert int(c.sum()) == math.comb(n, 3)


def test_balance_of_section_5_1():
    """Eq. 4 over the configurations of section 5.1 (units in multiples of 18
    from 18 to 522).  Recomputed, the paper's scheme peaks at 3.08 percent
    (order 3, 522 units), just above the stated 3; every other point is below
    it.  The tile dealing stays under 2 percent."""
    b = GOLD["balance"]
    worst_paper = worst_tiles = 0.0
    for k_s, n in b["variants_by_order"].items():
        k = int(k_s)
        for p in range(b["units_min"], b["units_max"] + 1, 18):
            e0 = imbalance(fiuncho.shard_counts(n, 2048, k, p, fiuncho.PREFIX_ROUND_ROBIN), n, k)
            e1 = imbalance(fiuncho.shard_counts(n, 2048, k, p, fiuncho.TILE_ROUND_ROBIN), n, k)
            if (k, p) != (3, 522):
                assert e0 < b["stated_max_percent"], (k, p, e0)
            worst_paper = max(worst_paper, e0)
            worst_tiles = max(worst_tiles, e1)
    assert 3.0 < worst_paper < 3.1
    assert worst_tiles < 2.0


def test_shard_counts_errors():
    L = fiuncho.lib()
    buf = np.zeros(4, np.uint64)
    assert L.fiuncho_shard_counts(10, 64, 2, 4, 0, None) == fiuncho.E_NULL
    assert L.fiuncho_shard_counts(10, 64, 2, 0, 0, buf.ctypes.data) == fiuncho.E_SHAPE
    assert L.fiuncho_shard_counts(10, 64, 2, 4, 2, buf.ctypes.data) == fiuncho.E_SHAPE
    assert L.fiuncho_shard_counts(0, 64, 1, 4, 0, buf.ctypes.data) == fiuncho.E_SHAPE
    assert L.fiuncho_shard_counts(10, 64, 9, 4, 0, buf.ctypes.data) == fiuncho.E_ORDER
    assert L.fiuncho_shard_counts(3, 64, 4, 4, 1, buf.ctypes.data) == fiuncho.E_ORDER
    assert L.fiuncho_shard_counts(1 << 20, 64, 8, 4, 0, buf.ctypes.data) == fiuncho.E_OVERFLOW


def test_job_shard_index_checked_on_host():
    jobs = (fiuncho.Job * 1)()
    jobs[0].snps, jobs[0].samples, jobs[0].order, jobs[0].top_n = 50, 64, 2, 5
    jobs[0].shard_index, jobs[0].shard_count = 3, 3
    assert fiuncho.lib().fiuncho_workspace_bytes(jobs, 1) == 0
    assert "shard_index" in fiuncho.last_error()
    jobs[0].shard_index = 2
    assert fiuncho.lib().fiuncho_workspace_bytes(jobs, 1) > 0
