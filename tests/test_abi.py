"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid input on the host before any device work
(no GPU is touched by these tests)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2201_03331_amd import fiuncho

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fiuncho.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fiuncho_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fiuncho.lib()
    decl = declared_functions()
    assert decl == sorted(fiuncho.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def test_hit_layout_matches_header():
    # snp[8] (32 B) + rank (8 B) + mi (8 B) + mi32, rel_err, est, reserved (16 B)
    assert fiuncho.HIT_DTYPE.itemsize == 64
    assert [fiuncho.HIT_DTYPE.fields[f][1] for f in ("snp", "rank", "mi", "mi32", "rel_err", "est")] == \
        [0, 32, 40, 48, 52, 56]
    assert ctypes.sizeof(fiuncho.Job) == 64
    assert ctypes.sizeof(fiuncho.Profile) == 56


def test_estimate_bound():
    """u (6 ln m + (3^k + 4) ln 2) with u = 2^-24 (the rounding bound of the
    plain single-precision evaluation of Eq. 1-3); negative for invalid
    arguments.  Host-only."""
    import math
    u = 2.0 ** -24
    for k, m in ((1, 1), (2, 1600), (3, 6400), (5, 4000), (8, (1 << 24) - 1)):
        want = u * (6 * math.log(m) + (3 ** k + 4) * math.log(2))
        assert fiuncho.estimate_bound(k, m) == pytest.approx(want, rel=1e-12)
    assert fiuncho.estimate_bound(0, 10) < 0
    assert fiuncho.estimate_bound(9, 10) < 0
    assert fiuncho.estimate_bound(2, 0) < 0


def _data(n=6, m=40, seed=0):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 3, (n, m), dtype=np.uint8), (rng.random(m) < 0.5).astype(np.uint8)


def test_host_validation_codes():
    G, y = _data()
    Gb = G.copy()
    Gb[2, 5] = 3
    assert fiuncho.scan_code(Gb, y, 2, 5) == fiuncho.E_GENOTYPE
    assert "variant 2, sample 5" in fiuncho.last_error()
    yb = y.copy()
    yb[3] = 2
    assert fiuncho.scan_code(G, yb, 2, 5) == fiuncho.E_PHENOTYPE
    assert fiuncho.scan_code(G, y, 0, 5) == fiuncho.E_ORDER
    assert fiuncho.scan_code(G, y, 7, 5) == fiuncho.E_ORDER
    assert fiuncho.scan_code(G, y, 9, 5) == fiuncho.E_ORDER
    assert fiuncho.scan_code(G, y, 2, 0) == fiuncho.E_TOPN
    assert fiuncho.scan_code(G, y, 2, fiuncho.MAX_TOPN + 1) == fiuncho.E_TOPN


def test_overflow_and_shape_codes():
    # C(2^20, 8) does not fit in 63 bits; samples is irrelevant to the check
    big = np.zeros((1, 1), np.uint8)
    L = fiuncho.lib()
    n_out = ctypes.c_uint32(0)
    out = np.zeros(4, fiuncho.HIT_DTYPE)
    y = np.zeros(1, np.uint8)
    code = L.fiuncho_scan(big.ctypes.data, y.ctypes.data, 1 << 20, 1, 8, 4, out.ctypes.data,
                          ctypes.byref(n_out))
    assert code == fiuncho.E_OVERFLOW
    code = L.fiuncho_scan(big.ctypes.data, y.ctypes.data, 4, 1 << 24, 2, 4, out.ctypes.data,
                          ctypes.byref(n_out))
    assert code == fiuncho.E_SHAPE
    code = L.fiuncho_scan(None, y.ctypes.data, 4, 4, 2, 4, out.ctypes.data, ctypes.byref(n_out))
    assert code == fiuncho.E_NULL


def test_workspace_bytes_depends_on_shape_only():
    a = fiuncho.workspace_bytes([(100, 1600, 2, 10)])
    b = fiuncho.workspace_bytes([(100, 1600, 2, 10)])
    c = fiuncho.workspace_bytes([(100, 1600, 2, 10), (50, 999, 3, 7)])
    assert a == b > 0 and c > a
    assert fiuncho.workspace_bytes([(100, 1600, 0, 10)]) == 0


def test_static_scratch_rejects_large_jobs():
    """fiuncho_scan_batch_static refuses, before any device work, jobs whose
    workspace exceeds its static scratch.  Host-only."""
    assert fiuncho.STATIC_SCRATCH_BYTES == 64 << 20
    arr = fiuncho._job_shapes([(2000, 6400, 3, 100)])
    assert fiuncho.lib().fiuncho_workspace_bytes(arr, 1) > fiuncho.STATIC_SCRATCH_BYTES
    code = fiuncho.lib().fiuncho_scan_batch_static(arr, 1, fiuncho.DEVICE_PTRS, None)
    assert code == fiuncho.E_WORKSPACE
    assert "static scratch holds 67108864" in fiuncho.last_error()
    assert fiuncho.lib().fiuncho_scan_batch_static(None, 0, fiuncho.DEVICE_PTRS, None) == fiuncho.E_NULL


def test_contingency_rejects_bad_rank():
    G, y = _data()
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.contingency(G, y, 2, [15])   # C(6, 2) = 15
    assert e.value.code == fiuncho.E_SHAPE


def test_no_cpu_fallback_in_product():
    """The product package never imports or calls the reference."""
    pkg = os.path.join(ROOT, "paper_2201_03331_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f


def test_kernel_choice_table(monkeypatch):
    """The kernel each shape gets: built-in rule, table entries set and
    cleared per (order, snps, words) bucket, environment overrides first;
    the tile dealing follows the chosen kernel.  Host-only."""
    monkeypatch.delenv("FIUNCHO_ORDER2_MFMA", raising=False)
    monkeypatch.delenv("FIUNCHO_ORDER3_PAIRS", raising=False)
    monkeypatch.delenv("FIUNCHO_ORDER4_TRIPLES", raising=False)
    monkeypatch.delenv("FIUNCHO_ORDER3_MFMA", raising=False)
    L = fiuncho.lib()
    assert fiuncho.get_kernel(100, 1600, 2) == fiuncho.KERNEL_MFMA_FP4
    assert fiuncho.get_kernel(4000, 16000, 2) == fiuncho.KERNEL_MFMA_FP4
    assert fiuncho.get_kernel(1000, 6400, 2) == fiuncho.KERNEL_POPCOUNT  # 100 words
    assert fiuncho.get_kernel(1000, 9000, 2) == fiuncho.KERNEL_MFMA_FP4  # 141 words
    assert fiuncho.get_kernel(5000, 1000, 2) == fiuncho.KERNEL_MFMA_FP4
    assert fiuncho.get_kernel(1000, 6400, 3) == fiuncho.KERNEL_MFMA_FP4
    assert fiuncho.get_kernel(3, 10, 3) == fiuncho.KERNEL_MFMA_FP4
    assert fiuncho.get_kernel(300, 17000, 2) == fiuncho.KERNEL_MFMA_FP4  # 266 words
    assert fiuncho.get_kernel(200, 4000, 4) == fiuncho.KERNEL_MFMA_FP4_TABLES
    assert fiuncho.get_kernel(200, 16384, 4) == fiuncho.KERNEL_TRIPLES  # packed tables: below 16,384
    assert fiuncho.get_kernel(800, 4000, 4) == fiuncho.KERNEL_MFMA_FP4_TABLES  # 9.2 GB packed tables
    assert fiuncho.get_kernel(800, 17000, 4) == fiuncho.KERNEL_MFMA_FP4  # unpacked tables over 16 GiB
    assert fiuncho.get_kernel(5000, 4000, 4) == fiuncho.KERNEL_MFMA_FP4  # tables over 16 GiB
    assert fiuncho.get_kernel(5000, 30000, 4) == fiuncho.KERNEL_POPCOUNT  # over 20,447 samples
    assert fiuncho.get_kernel(100, 4000, 5) == fiuncho.KERNEL_MFMA_FP4_TABLES
    assert fiuncho.get_kernel(100, 16384, 5) == fiuncho.KERNEL_MFMA_FP4  # packed tables: below 16,384
    assert fiuncho.get_kernel(700, 4000, 5) == fiuncho.KERNEL_MFMA_FP4  # quad tables over 48 GiB
    assert fiuncho.get_kernel(100, 20448, 5) == fiuncho.KERNEL_POPCOUNT
    assert fiuncho.get_kernel(100, 4000, 6) == fiuncho.KERNEL_POPCOUNT
    assert L.fiuncho_get_kernel(5, 100, 6) == fiuncho.E_ORDER
    before = fiuncho.shard_counts(300, 500, 2, 5, fiuncho.TILE_ROUND_ROBIN)
    try:
        fiuncho.set_kernel(300, 500, 2, fiuncho.KERNEL_MFMA)
        assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_MFMA
        # same bucket (bit lengths of snps and of words), other sizes
        assert fiuncho.get_kernel(400, 450, 2) == fiuncho.KERNEL_MFMA
        assert fiuncho.get_kernel(600, 500, 2) == fiuncho.KERNEL_POPCOUNT
        after = fiuncho.shard_counts(300, 500, 2, 5, fiuncho.TILE_ROUND_ROBIN)
        assert int(after.sum()) == int(before.sum()) and after.tolist() != before.tolist()
        monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "0")
        assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_POPCOUNT
        monkeypatch.setenv("FIUNCHO_ORDER2_MFMA", "4")
        assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_MFMA_FP4
        monkeypatch.delenv("FIUNCHO_ORDER2_MFMA")
        monkeypatch.setenv("FIUNCHO_ORDER3_MFMA", "4")
        assert fiuncho.get_kernel(300, 500, 3) == fiuncho.KERNEL_MFMA_FP4
        monkeypatch.delenv("FIUNCHO_ORDER3_MFMA")
        # the operand format does not change the tile dealing
        fiuncho.set_kernel(300, 500, 2, fiuncho.KERNEL_MFMA_FP4)
        assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_MFMA_FP4
        assert fiuncho.shard_counts(300, 500, 2, 5, fiuncho.TILE_ROUND_ROBIN).tolist() == after.tolist()
    finally:
        fiuncho.set_kernel(300, 500, 2, fiuncho.KERNEL_AUTO)
    assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_POPCOUNT
    assert L.fiuncho_set_kernel(300, 500, 4, fiuncho.KERNEL_MFMA) == fiuncho.E_SHAPE
    assert L.fiuncho_set_kernel(300, 500, 6, fiuncho.KERNEL_MFMA_FP4) == fiuncho.E_SHAPE
    assert L.fiuncho_set_kernel(4, 500, 5, fiuncho.KERNEL_MFMA_FP4) == fiuncho.E_ORDER
    assert L.fiuncho_set_kernel(2, 500, 3, fiuncho.KERNEL_MFMA_FP4) == fiuncho.E_ORDER
    assert L.fiuncho_set_kernel(300, 500, 2, fiuncho.KERNEL_PAIRS) == fiuncho.E_SHAPE
    assert L.fiuncho_set_kernel(300, 500, 2, 9) == fiuncho.E_SHAPE
    assert L.fiuncho_set_kernel(300, 500, 3, fiuncho.KERNEL_TRIPLES) == fiuncho.E_SHAPE
    assert L.fiuncho_set_kernel(5000, 500, 4, fiuncho.KERNEL_TRIPLES) == fiuncho.E_SHAPE
    k = ctypes.c_int(0)
    assert L.fiuncho_autotune(300, 500, 2, 1, None) == fiuncho.E_NULL
    # launch configurations: kernel and waves per SIMD per bucket
    try:
        assert fiuncho.get_config(300, 500, 2) == (fiuncho.KERNEL_POPCOUNT, 0)
        fiuncho.set_config(300, 500, 2, fiuncho.KERNEL_MFMA_FP4, 2)
        assert fiuncho.get_config(300, 500, 2) == (fiuncho.KERNEL_MFMA_FP4, 2)
        assert fiuncho.get_config(400, 450, 2) == (fiuncho.KERNEL_MFMA_FP4, 2)  # same bucket
        assert fiuncho.get_kernel(300, 500, 2) == fiuncho.KERNEL_MFMA_FP4
        fiuncho.set_kernel(300, 500, 2, fiuncho.KERNEL_MFMA)   # set_kernel: waves per SIMD 0
        assert fiuncho.get_config(300, 500, 2) == (fiuncho.KERNEL_MFMA, 0)
        assert L.fiuncho_set_config(300, 500, 2, fiuncho.KERNEL_MFMA, 9) == fiuncho.E_SHAPE
        assert L.fiuncho_set_config(300, 500, 2, fiuncho.KERNEL_MFMA, -1) == fiuncho.E_SHAPE
        assert L.fiuncho_set_config(300, 500, 2, fiuncho.KERNEL_PAIRS, 1) == fiuncho.E_SHAPE
        assert L.fiuncho_get_config(300, 500, 2, None, None) == fiuncho.E_NULL
        assert L.fiuncho_get_config(3, 500, 4, ctypes.byref(k), ctypes.byref(k)) == fiuncho.E_ORDER
    finally:
        fiuncho.set_config(300, 500, 2, fiuncho.KERNEL_AUTO, 0)
    assert fiuncho.get_config(300, 500, 2) == (fiuncho.KERNEL_POPCOUNT, 0)
    assert L.fiuncho_autotune(3, 500, 4, 1, ctypes.byref(k)) == fiuncho.E_ORDER


def test_build_checks_lds_window_kernels_have_no_static_lds():
    # the FP4 matrix-core kernels read their f table from LDS address 0, which
    # holds only while they declare no static LDS; the build parses the
    # compiler's resource remarks and refuses a library where one does
    from paper_2201_03331_amd import build
    name = "_ZN7fiuncho11mfma_kernelILi3ELi3EEEvNS_7GlobalsE"
    ok = (f"mfma.hip:1:1: remark: Function Name: {name} [-Rpass-analysis=kernel-resource-usage]\n"
          "mfma.hip:1:1: remark:     LDS Size [bytes/block]: 0 [-Rpass-analysis=kernel-resource-usage]\n")
    build.check_lds_window(ok)
    with pytest.raises(RuntimeError, match="static LDS"):
        build.check_lds_window(ok.replace("block]: 0", "block]: 8"))
    with pytest.raises(RuntimeError, match="no resource remarks"):
        build.check_lds_window(ok.replace(name, "_ZN7fiuncho13select_kernelEv"))
    # the int8 kernel keeps its static byte table and is not checked
    assert not build.LDS_WINDOW_KERNELS.match("_ZN7fiuncho11mfma_kernelILi3ELi0EEEvNS_7GlobalsE")
