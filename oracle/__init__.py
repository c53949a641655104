"""ctypes wrapper around ``oracle.c``: the plain CPU reference of the scan.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP implementation.

Every function follows the paper's definitions:
  * ``table``      -- contingency table of one combination (section 3.2,
                      Fig. 3), counted one sample at a time;
  * ``mi``         -- mutual information of a table (section 3.3, Eq. 1-3);
  * ``scan``       -- the exhaustive search of Fig. 1 / Algorithm 1 keeping the
                      best ``top_n`` under (MI descending, rank ascending);
  * ``rank``/``unrank``/``binom`` -- lexicographic numbering of combinations
                      (the enumeration order of Algorithm 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
BAD_ARG = -1
BAD_GENOTYPE = -3
BAD_PHENOTYPE = -4
BAD_ORDER = -5
BAD_TOPN = -6
OVERFLOW = -7

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_binom.restype = ctypes.c_uint64
        L.oracle_binom.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_rank.restype = ctypes.c_uint64
        L.oracle_rank.argtypes = [ctypes.c_uint32, ctypes.c_int, u32p]
        L.oracle_unrank.restype = None
        L.oracle_unrank.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64, u32p]
        L.oracle_validate.restype = ctypes.c_int
        L.oracle_validate.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int, ctypes.c_uint32]
        L.oracle_table.restype = None
        L.oracle_table.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_int, u32p, u32p]
        L.oracle_mi.restype = ctypes.c_double
        L.oracle_mi.argtypes = [u32p, ctypes.c_int]
        L.oracle_score_ranks.restype = ctypes.c_int
        L.oracle_score_ranks.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_int, u64p, ctypes.c_uint64, dp, u32p]
        L.oracle_scan_range.restype = ctypes.c_int
        L.oracle_scan_range.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int, u64p, dp, u32p]
        L.oracle_scan.restype = ctypes.c_int
        L.oracle_scan.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_int, ctypes.c_uint32, ctypes.c_int, u64p,
                                  dp, u32p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _arrays(G, y):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    assert G.ndim == 2 and y.ndim == 1 and G.shape[1] == y.shape[0]
    return G, y


def binom(n: int, k: int) -> int:
    """C(n, k); 2**64 - 1 when it does not fit in 64 bits."""
    return int(lib().oracle_binom(n, k))


def rank(n: int, comb) -> int:
    c = np.ascontiguousarray(comb, dtype=np.uint32)
    return int(lib().oracle_rank(n, len(c), _p(c, ctypes.c_uint32)))


def unrank(n: int, k: int, r: int) -> tuple:
    c = np.zeros(k, dtype=np.uint32)
    lib().oracle_unrank(n, k, r, _p(c, ctypes.c_uint32))
    return tuple(int(v) for v in c)


def validate(G, y, k: int, top_n: int) -> int:
    G, y = _arrays(G, y)
    return int(lib().oracle_validate(_p(G, ctypes.c_uint8), _p(y, ctypes.c_uint8),
                                     G.shape[0], G.shape[1], k, top_n))


def table(G, y, comb) -> np.ndarray:
    """Contingency table of one combination: shape (3**k, 2), column = class."""
    G, y = _arrays(G, y)
    c = np.ascontiguousarray(comb, dtype=np.uint32)
    k = len(c)
    T = np.zeros((3 ** k, 2), dtype=np.uint32)
    lib().oracle_table(_p(G, ctypes.c_uint8), _p(y, ctypes.c_uint8), G.shape[0],
                       G.shape[1], k, _p(c, ctypes.c_uint32), _p(T, ctypes.c_uint32))
    return T


def mi(T) -> float:
    """Mutual information (nats) of a (3**k, 2) contingency table."""
    T = np.ascontiguousarray(T, dtype=np.uint32)
    cells = T.shape[0]
    k = 0
    while 3 ** k < cells:
        k += 1
    assert 3 ** k == cells
    return float(lib().oracle_mi(_p(T, ctypes.c_uint32), k))


def host_threads() -> int:
    """Host CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def score_ranks(G, y, k: int, ranks, want_tables: bool = False, nthreads: int = 0):
    """MI (and optionally tables) of the combinations with the given ranks.
    Long lists are split into contiguous parts scored by concurrent calls
    (``nthreads``; 0 = every host CPU); each rank is scored alone, so the
    values do not depend on the split."""
    G, y = _arrays(G, y)
    r = np.ascontiguousarray(ranks, dtype=np.uint64)
    mi_out = np.zeros(len(r), dtype=np.float64)
    tabs = np.zeros((len(r), 3 ** k, 2), dtype=np.uint32) if want_tables else None
    L = lib()

    def part(lo, hi):
        return L.oracle_score_ranks(
            _p(G, ctypes.c_uint8), _p(y, ctypes.c_uint8), G.shape[0], G.shape[1], k,
            _p(r[lo:hi], ctypes.c_uint64), hi - lo, _p(mi_out[lo:hi], ctypes.c_double),
            _p(tabs[lo:hi], ctypes.c_uint32) if want_tables else None)

    nt = nthreads if nthreads > 0 else host_threads()
    nt = max(1, min(nt, len(r) // 4096))
    if nt == 1:
        sts = [part(0, len(r))]
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = np.linspace(0, len(r), nt + 1).astype(np.int64)
        with ThreadPoolExecutor(nt) as ex:
            sts = list(ex.map(lambda i: part(int(cuts[i]), int(cuts[i + 1])), range(nt)))
    for st in sts:
        if st != OK:
            raise ValueError(f"oracle_score_ranks failed: {st}")
    return (mi_out, tabs) if want_tables else mi_out


def order_all(G, y, k: int, nthreads: int = 0):
    """Every combination of order k: (ranks, mi) in the output order (MI
    descending, rank ascending), each combination scored by the oracle."""
    total = binom(np.asarray(G).shape[0], k)
    ranks = np.arange(total, dtype=np.uint64)
    mi_all = score_ranks(G, y, k, ranks, nthreads=nthreads)
    order = np.lexsort((ranks, -mi_all))
    return ranks[order], mi_all[order]


def scan_range(G, y, k: int, top_n: int, first: int, count: int, nthreads: int = 0):
    """Best ``top_n`` of ranks [first, first+count): (ranks, mi) best first."""
    G, y = _arrays(G, y)
    if nthreads <= 0:
        nthreads = host_threads()
    cap = min(top_n, max(count, 1))
    out_r = np.zeros(cap, dtype=np.uint64)
    out_m = np.zeros(cap, dtype=np.float64)
    n_out = ctypes.c_uint32(0)
    st = lib().oracle_scan_range(
        _p(G, ctypes.c_uint8), _p(y, ctypes.c_uint8), G.shape[0], G.shape[1], k,
        top_n, first, count, nthreads, _p(out_r, ctypes.c_uint64),
        _p(out_m, ctypes.c_double), ctypes.byref(n_out))
    if st != OK:
        raise ValueError(f"oracle_scan_range failed: {st}")
    return out_r[: n_out.value].copy(), out_m[: n_out.value].copy()


def scan(G, y, k: int, top_n: int, nthreads: int = 0):
    """Whole exhaustive search: (ranks, mi) of the best ``top_n``, best first."""
    G, y = _arrays(G, y)
    return scan_range(G, y, k, top_n, 0, binom(G.shape[0], k), nthreads)
