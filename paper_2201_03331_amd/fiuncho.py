"""Python binding of libfiuncho.so (argument marshalling only).

Every step of the search runs in the library's gfx950 kernels; this module
loads the in-tree shared library, converts arguments and returns numpy arrays.
It fails loudly when the library is missing: there is no CPU fallback.
PyTorch is used only for device memory and streams (``DeviceBatch``).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfiuncho.so")

OK = 0
E_NULL = -1
E_SHAPE = -2
E_GENOTYPE = -3
E_PHENOTYPE = -4
E_ORDER = -5
E_TOPN = -6
E_OVERFLOW = -7
E_WORKSPACE = -8
E_DEVICE = -9
E_INTERNAL = -10
E_IO = -11
MAX_ORDER = 8
MAX_TOPN = 1 << 24
DEVICE_PTRS = 1
UPLOAD_PLAN = 2
STATIC_SCRATCH_BYTES = 64 << 20
KERNEL_AUTO = 0
KERNEL_POPCOUNT = 1
KERNEL_PAIRS = 2
KERNEL_MFMA = 3
KERNEL_TRIPLES = 4
KERNEL_MFMA_FP4 = 5
KERNEL_MFMA_FP4_TABLES = 6

# every entry point declared in include/fiuncho.h
EXPORTS = (
    "fiuncho_scan",
    "fiuncho_workspace_bytes",
    "fiuncho_scan_batch",
    "fiuncho_scan_batch_static",
    "fiuncho_contingency",
    "fiuncho_score",
    "fiuncho_shard_counts",
    "fiuncho_get_kernel",
    "fiuncho_set_kernel",
    "fiuncho_get_config",
    "fiuncho_set_config",
    "fiuncho_autotune",
    "fiuncho_last_error",
    "fiuncho_estimate_bound",
    "fiuncho_set_profiling",
    "fiuncho_get_profile",
    "fiuncho_read_genotypes",
    "fiuncho_read_phenotype",
    "fiuncho_write_hits",
)

HIT_DTYPE = np.dtype([("snp", "<u4", (MAX_ORDER,)), ("rank", "<u8"), ("mi", "<f8"),
                      ("mi32", "<f4"), ("rel_err", "<f4"), ("est", "<f4"), ("reserved", "<u4")])
assert HIT_DTYPE.itemsize == 64


class Job(ctypes.Structure):
    _fields_ = [
        ("genotypes", ctypes.c_void_p),
        ("phenotype", ctypes.c_void_p),
        ("snps", ctypes.c_uint32),
        ("samples", ctypes.c_uint32),
        ("order", ctypes.c_int),
        ("top_n", ctypes.c_uint32),
        ("out", ctypes.c_void_p),
        ("n_out", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("shard_index", ctypes.c_uint32),
        ("shard_count", ctypes.c_uint32),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("pack_ms", ctypes.c_float),
        ("pilot_ms", ctypes.c_float),
        ("scan_ms", ctypes.c_float),
        ("mfma_ms", ctypes.c_float),
        ("select_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
        ("calls", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("combinations", ctypes.c_uint64),
        ("candidates", ctypes.c_uint64),
        ("kept", ctypes.c_uint32),
        ("kernels", ctypes.c_uint32),
    ]


class FiunchoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fiuncho error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname; loading it
        # first makes this library bind to it, so that torch tensors, torch
        # streams and these kernels share one runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2201_03331_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.c_void_p
        L.fiuncho_scan.restype = ctypes.c_int
        L.fiuncho_scan.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]
        L.fiuncho_workspace_bytes.restype = ctypes.c_size_t
        L.fiuncho_workspace_bytes.argtypes = [ctypes.POINTER(Job), ctypes.c_uint32]
        L.fiuncho_scan_batch.restype = ctypes.c_int
        L.fiuncho_scan_batch.argtypes = [ctypes.POINTER(Job), ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fiuncho_scan_batch_static.restype = ctypes.c_int
        L.fiuncho_scan_batch_static.argtypes = [ctypes.POINTER(Job), ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_void_p]
        L.fiuncho_contingency.restype = ctypes.c_int
        L.fiuncho_contingency.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.fiuncho_score.restype = ctypes.c_int
        L.fiuncho_score.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]
        L.fiuncho_shard_counts.restype = ctypes.c_int
        L.fiuncho_shard_counts.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                           ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        L.fiuncho_get_kernel.restype = ctypes.c_int
        L.fiuncho_get_kernel.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        L.fiuncho_set_kernel.restype = ctypes.c_int
        L.fiuncho_set_kernel.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
        L.fiuncho_get_config.restype = ctypes.c_int
        L.fiuncho_get_config.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.fiuncho_set_config.restype = ctypes.c_int
        L.fiuncho_set_config.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int]
        L.fiuncho_autotune.restype = ctypes.c_int
        L.fiuncho_autotune.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_int)]
        L.fiuncho_last_error.restype = ctypes.c_char_p
        L.fiuncho_last_error.argtypes = []
        L.fiuncho_estimate_bound.restype = ctypes.c_double
        L.fiuncho_estimate_bound.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.fiuncho_set_profiling.restype = None
        L.fiuncho_set_profiling.argtypes = [ctypes.c_int]
        L.fiuncho_get_profile.restype = ctypes.c_int
        L.fiuncho_get_profile.argtypes = [ctypes.POINTER(Profile)]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.fiuncho_read_genotypes.restype = ctypes.c_int
        L.fiuncho_read_genotypes.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_size_t, u32p, u32p]
        L.fiuncho_read_phenotype.restype = ctypes.c_int
        L.fiuncho_read_phenotype.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_size_t, u32p]
        L.fiuncho_write_hits.restype = ctypes.c_int
        L.fiuncho_write_hits.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().fiuncho_last_error().decode()


def estimate_bound(order: int, samples: int) -> float:
    """Bound of |est - mi| for this order and sample count
    (fiuncho_estimate_bound)."""
    return float(lib().fiuncho_estimate_bound(order, samples))


def _check(code: int):
    if code != OK:
        raise FiunchoError(code, last_error())


def read_genotypes(path) -> np.ndarray:
    """[snps][samples] uint8 genotypes of a genotype text file
    (fiuncho_read_genotypes: measured, then read)."""
    L, p = lib(), os.fsencode(path)
    n, m = ctypes.c_uint32(), ctypes.c_uint32()
    _check(L.fiuncho_read_genotypes(p, None, 0, ctypes.byref(n), ctypes.byref(m)))
    G = np.empty((n.value, m.value), dtype=np.uint8)
    _check(L.fiuncho_read_genotypes(p, G.ctypes.data, G.nbytes, ctypes.byref(n), ctypes.byref(m)))
    return G


def read_phenotype(path) -> np.ndarray:
    """[samples] uint8 classes of a phenotype text file (fiuncho_read_phenotype)."""
    L, p = lib(), os.fsencode(path)
    m = ctypes.c_uint32()
    _check(L.fiuncho_read_phenotype(p, None, 0, ctypes.byref(m)))
    y = np.empty(m.value, dtype=np.uint8)
    _check(L.fiuncho_read_phenotype(p, y.ctypes.data, y.nbytes, ctypes.byref(m)))
    return y


def read_dataset(genotype_path, phenotype_path):
    """(G, y) from a genotype and a phenotype file; ValueError if their sample
    counts differ."""
    G, y = read_genotypes(genotype_path), read_phenotype(phenotype_path)
    if G.shape[1] != y.shape[0]:
        raise ValueError(f"{G.shape[1]} samples in {genotype_path}, {y.shape[0]} in {phenotype_path}")
    return G, y


def write_hits(path, hits: np.ndarray, order: int) -> None:
    """Writes hits (HIT_DTYPE, best first) to a result file (fiuncho_write_hits)."""
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    _check(lib().fiuncho_write_hits(os.fsencode(path), hits.ctypes.data if len(hits) else None, len(hits),
                                    order))


def _host_arrays(G, y):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    if G.ndim != 2 or y.ndim != 1 or G.shape[1] != y.shape[0]:
        raise ValueError("genotypes must be [snps][samples] and phenotype [samples]")
    return G, y


def scan(G, y, order: int, top_n: int) -> np.ndarray:
    """Exhaustive search on host arrays (fiuncho_scan); hits best first."""
    G, y = _host_arrays(G, y)
    k = order
    room = min(top_n, math.comb(G.shape[0], k)) if 1 <= k <= G.shape[0] else 1
    out = np.zeros(max(room, 1), dtype=HIT_DTYPE)
    n_out = ctypes.c_uint32(0)
    _check(lib().fiuncho_scan(G.ctypes.data, y.ctypes.data, G.shape[0], G.shape[1], order, top_n,
                              out.ctypes.data, ctypes.byref(n_out)))
    return out[: n_out.value]


def scan_code(G, y, order: int, top_n: int) -> int:
    """Return code of fiuncho_scan (for error-path checks)."""
    G = np.ascontiguousarray(G, dtype=np.uint8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    n = G.shape[0] if G.ndim == 2 else 0
    m = G.shape[1] if G.ndim == 2 else 0
    # room for what a successful call writes: min(top_n, C(n, order)) hits
    room = min(top_n, math.comb(n, order)) if 1 <= order <= n else 1
    out = np.zeros(max(room, 1), dtype=HIT_DTYPE)
    n_out = ctypes.c_uint32(7)
    code = lib().fiuncho_scan(G.ctypes.data, y.ctypes.data, n, m, order, top_n, out.ctypes.data,
                              ctypes.byref(n_out))
    if code != OK:
        assert n_out.value == 0
    return code


def contingency(G, y, order: int, ranks) -> np.ndarray:
    """Contingency tables [len(ranks)][3**order][2] (fiuncho_contingency)."""
    G, y = _host_arrays(G, y)
    r = np.ascontiguousarray(ranks, dtype=np.uint64)
    tabs = np.zeros((len(r), 3 ** order, 2), dtype=np.uint32)
    _check(lib().fiuncho_contingency(G.ctypes.data, y.ctypes.data, G.shape[0], G.shape[1], order,
                                     r.ctypes.data, len(r), tabs.ctypes.data))
    return tabs


def score(G, y, order: int, ranks):
    """(est, mi32, mi) of explicit combinations (fiuncho_score)."""
    G, y = _host_arrays(G, y)
    r = np.ascontiguousarray(ranks, dtype=np.uint64)
    est = np.zeros(len(r), dtype=np.float32)
    m32 = np.zeros(len(r), dtype=np.float32)
    m64 = np.zeros(len(r), dtype=np.float64)
    _check(lib().fiuncho_score(G.ctypes.data, y.ctypes.data, G.shape[0], G.shape[1], order,
                               r.ctypes.data, len(r), est.ctypes.data, m32.ctypes.data,
                               m64.ctypes.data))
    return est, m32, m64


PREFIX_ROUND_ROBIN = 0
TILE_ROUND_ROBIN = 1


def shard_counts(snps: int, samples: int, order: int, units: int,
                 scheme: int = PREFIX_ROUND_ROBIN) -> np.ndarray:
    """Combinations per processing unit under a static distribution
    (fiuncho_shard_counts; host-only)."""
    counts = np.zeros(units, dtype=np.uint64)
    _check(lib().fiuncho_shard_counts(snps, samples, order, units, scheme, counts.ctypes.data))
    return counts


def get_kernel(snps: int, samples: int, order: int) -> int:
    """KERNEL_* value a job of this shape would use (fiuncho_get_kernel)."""
    k = lib().fiuncho_get_kernel(snps, samples, order)
    if k < 0:
        raise FiunchoError(k, last_error())
    return k


def set_kernel(snps: int, samples: int, order: int, kernel: int):
    _check(lib().fiuncho_set_kernel(snps, samples, order, kernel))


def get_config(snps: int, samples: int, order: int):
    """(KERNEL_* value, waves per SIMD) a job of this shape would use
    (fiuncho_get_config; waves per SIMD 0 = as many as fit)."""
    k, w = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().fiuncho_get_config(snps, samples, order, ctypes.byref(k), ctypes.byref(w)))
    return k.value, w.value


def set_config(snps: int, samples: int, order: int, kernel: int, waves_per_simd: int = 0):
    _check(lib().fiuncho_set_config(snps, samples, order, kernel, waves_per_simd))


def autotune(snps: int, samples: int, order: int, reps: int = 3) -> int:
    """Times the kernels for this shape on the device and records the fastest
    (fiuncho_autotune); returns its KERNEL_* value."""
    k = ctypes.c_int(0)
    _check(lib().fiuncho_autotune(snps, samples, order, reps, ctypes.byref(k)))
    return k.value


def set_profiling(enable: bool):
    lib().fiuncho_set_profiling(1 if enable else 0)


def get_profile() -> dict:
    p = Profile()
    _check(lib().fiuncho_get_profile(ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in Profile._fields_}


def _job_shapes(shapes):
    arr = (Job * len(shapes))()
    for i, (n, m, k, top) in enumerate(shapes):
        arr[i].snps, arr[i].samples, arr[i].order, arr[i].top_n = n, m, k, top
    return arr


def workspace_bytes(shapes) -> int:
    """Workspace for jobs given as (snps, samples, order, top_n) tuples."""
    arr = _job_shapes(shapes)
    return int(lib().fiuncho_workspace_bytes(arr, len(shapes)))


class DeviceBatch:
    """Inputs, outputs and workspace of a batched search held in device memory
    (torch tensors); ``run`` queues fiuncho_scan_batch on a stream."""

    def __init__(self, datasets, device="cuda", shards=None):
        """``shards``: optional (shard_index, shard_count) per dataset."""
        import torch

        self.torch = torch
        self.shapes = [(d.n, d.m, d.order, d.top_n) for d in datasets]
        self.G = [torch.from_numpy(np.ascontiguousarray(d.genotypes)).to(device) for d in datasets]
        self.y = [torch.from_numpy(np.ascontiguousarray(d.phenotype)).to(device) for d in datasets]
        self.out = [torch.zeros(d.top_n * HIT_DTYPE.itemsize, dtype=torch.uint8, device=device)
                    for d in datasets]
        self.n_out = torch.zeros(len(datasets), dtype=torch.int32, device=device)
        self.status = torch.zeros(len(datasets), dtype=torch.int32, device=device)
        self.jobs = (Job * len(datasets))()
        for i, d in enumerate(datasets):
            J = self.jobs[i]
            J.genotypes = self.G[i].data_ptr()
            J.phenotype = self.y[i].data_ptr()
            J.snps, J.samples, J.order, J.top_n = d.n, d.m, d.order, d.top_n
            J.out = self.out[i].data_ptr()
            J.n_out = self.n_out.data_ptr() + 4 * i
            J.status = self.status.data_ptr() + 4 * i
            if shards is not None:
                J.shard_index, J.shard_count = shards[i]
        self.ws_bytes = int(lib().fiuncho_workspace_bytes(self.jobs, len(datasets)))
        if self.ws_bytes == 0:
            raise FiunchoError(E_SHAPE, last_error())
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        # a new workspace may reuse the memory of one the library planned
        # before (the caching allocator hands back freed blocks), which other
        # tensors may have overwritten since: the first run uploads the plan
        self._planned = False

    def run(self, stream=None, upload_plan: bool = False):
        s = stream if stream is not None else self.torch.cuda.current_stream()
        flags = DEVICE_PTRS | (UPLOAD_PLAN if upload_plan or not self._planned else 0)
        _check(lib().fiuncho_scan_batch(self.jobs, len(self.shapes), flags, self.ws_ptr,
                                        self.ws_bytes, s.cuda_stream))
        self._planned = True

    def run_static(self, stream=None):
        """Queues fiuncho_scan_batch_static (the library's static scratch
        instead of this batch's workspace; no device allocation)."""
        s = stream if stream is not None else self.torch.cuda.current_stream()
        _check(lib().fiuncho_scan_batch_static(self.jobs, len(self.shapes), DEVICE_PTRS, s.cuda_stream))

    def capture(self, profile: bool = False):
        """Capture one ``run`` into a HIP graph (torch.cuda.CUDAGraph).  The
        first eager ``run`` uploads the plan; the captured call then queues
        kernels only (no allocation, no memset, no host synchronisation).
        With ``profile`` the phase events are captured too, so that
        ``get_profile`` after replays reports the last replay."""
        torch = self.torch
        self.run()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        if profile:
            set_profiling(True)
        with torch.cuda.graph(self.graph):
            self.run(torch.cuda.current_stream())
        if profile:
            set_profiling(False)
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()

    def results(self):
        """Per job: (status, hits) after the stream has finished."""
        self.torch.cuda.synchronize()
        n_out = self.n_out.cpu().numpy()
        status = self.status.cpu().numpy()
        res = []
        for i in range(len(self.shapes)):
            raw = self.out[i].cpu().numpy()
            hits = raw.view(HIT_DTYPE)[: int(n_out[i])].copy()
            res.append((int(status[i]), hits))
        return res
