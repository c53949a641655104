"""The input and output stages (Fig. 1: variants read from a file, the saved
combinations written to one): the library's text reader and writer, on the
host (no GPU needed), and the whole program read -> search -> write on the
GPU against the oracle."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_2201_03331_amd import fiuncho
from paper_2201_03331_amd.__main__ import main


def write_text(path, text):
    with open(path, "w", newline="") as f:
        f.write(text)


def dataset(seed, n, m):
    rng = np.random.default_rng(seed)
    G = rng.integers(0, 3, size=(n, m), dtype=np.uint8)
    y = rng.integers(0, 2, size=m, dtype=np.uint8)
    return G, y


@pytest.mark.parametrize("style", ["compact", "spaces", "tabs", "commas", "crlf"])
def test_read_round_trip(tmp_path, style):
    G, y = dataset(1, 37, 101)
    sep = {"compact": "", "spaces": " ", "tabs": "\t", "commas": ",", "crlf": " "}[style]
    nl = "\r\n" if style == "crlf" else "\n"
    lines = ["# variants of a test", ""] + [sep.join(str(v) for v in row) for row in G]
    write_text(tmp_path / "g.txt", nl.join(lines) + nl + nl)
    # the phenotype over several lines, with a comment
    half = len(y) // 2
    write_text(tmp_path / "y.txt", "# classes" + nl + sep.join(map(str, y[:half])) + nl +
               sep.join(map(str, y[half:])))
    G2, y2 = fiuncho.read_dataset(tmp_path / "g.txt", tmp_path / "y.txt")
    np.testing.assert_array_equal(G2, G)
    np.testing.assert_array_equal(y2, y)


def test_read_errors(tmp_path):
    write_text(tmp_path / "ragged.txt", "0120\n012\n")
    write_text(tmp_path / "bad.txt", "0120\n0130\n")
    write_text(tmp_path / "empty.txt", "# nothing\n\n")
    write_text(tmp_path / "y.txt", "0 1 2\n")
    write_text(tmp_path / "y3.txt", "0 1 1\n")
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.read_genotypes(tmp_path / "ragged.txt")
    assert e.value.code == fiuncho.E_SHAPE and "line 2" in str(e.value)
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.read_genotypes(tmp_path / "bad.txt")
    assert e.value.code == fiuncho.E_GENOTYPE and "line 2" in str(e.value)
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.read_genotypes(tmp_path / "empty.txt")
    assert e.value.code == fiuncho.E_SHAPE
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.read_genotypes(tmp_path / "missing.txt")
    assert e.value.code == fiuncho.E_IO
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.read_phenotype(tmp_path / "y.txt")
    assert e.value.code == fiuncho.E_PHENOTYPE
    # a buffer smaller than the file's matrix is refused before anything is written
    L = fiuncho.lib()
    n, m = ctypes.c_uint32(), ctypes.c_uint32()
    buf = (ctypes.c_uint8 * 3)()
    write_text(tmp_path / "g.txt", "0120\n1201\n")
    assert L.fiuncho_read_genotypes(os.fsencode(tmp_path / "g.txt"), ctypes.addressof(buf), 3,
                                    ctypes.byref(n), ctypes.byref(m)) == fiuncho.E_SHAPE
    assert L.fiuncho_read_genotypes(None, None, 0, ctypes.byref(n), ctypes.byref(m)) == fiuncho.E_NULL
    assert L.fiuncho_read_phenotype(os.fsencode(tmp_path / "y3.txt"), ctypes.addressof(buf), 2,
                                    ctypes.byref(m)) == fiuncho.E_SHAPE
    # samples counts of the two files differ
    write_text(tmp_path / "y2.txt", "0 1\n")
    with pytest.raises(ValueError):
        fiuncho.read_dataset(tmp_path / "g.txt", tmp_path / "y2.txt")


def parse_result(path, order):
    lines = open(path).read().splitlines()
    head = lines[0].split("\t")
    assert head == ["rank"] + [f"snp{i + 1}" for i in range(order)] + ["mi", "mi32", "rel_err", "est"]
    rows = [l.split("\t") for l in lines[1:]]
    ranks = np.array([int(r[0]) for r in rows], dtype=np.uint64)
    snps = np.array([[int(v) for v in r[1:1 + order]] for r in rows], dtype=np.uint32).reshape(-1, order)
    mi = np.array([float(r[1 + order]) for r in rows])
    return ranks, snps, mi


def test_write_round_trip(tmp_path):
    rng = np.random.default_rng(3)
    hits = np.zeros(5, dtype=fiuncho.HIT_DTYPE)
    hits["snp"][:, :3] = np.sort(rng.choice(1000, size=(5, 3), replace=False), axis=1)
    hits["snp"][:, 3:] = 0xFFFFFFFF
    hits["rank"] = rng.integers(0, 10 ** 12, size=5)
    hits["mi"] = rng.random(5) * 1e-2
    hits["mi32"] = hits["mi"].astype(np.float32)
    fiuncho.write_hits(tmp_path / "r.tsv", hits, 3)
    ranks, snps, mi = parse_result(tmp_path / "r.tsv", 3)
    np.testing.assert_array_equal(ranks, hits["rank"])
    np.testing.assert_array_equal(snps, hits["snp"][:, :3])
    np.testing.assert_array_equal(mi, hits["mi"])  # 17 significant digits: exact
    fiuncho.write_hits(tmp_path / "empty.tsv", hits[:0], 2)
    assert open(tmp_path / "empty.tsv").read().splitlines() == ["rank\tsnp1\tsnp2\tmi\tmi32\trel_err\test"]
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.write_hits(tmp_path / "r.tsv", hits, 0)
    assert e.value.code == fiuncho.E_ORDER
    with pytest.raises(fiuncho.FiunchoError) as e:
        fiuncho.write_hits(tmp_path / "no_such_dir" / "r.tsv", hits, 3)
    assert e.value.code == fiuncho.E_IO


@pytest.mark.gpu
@pytest.mark.parametrize("order,n,m,top_n", [(2, 60, 301, 15), (3, 30, 257, 10)])
def test_program_read_search_write(tmp_path, order, n, m, top_n):
    """Fig. 1 end to end: files in, the search on the GPU, the result file out;
    the result file holds the oracle's best combinations with their exact MI."""
    G, y = dataset(40 + order, n, m)
    write_text(tmp_path / "g.txt", "\n".join(" ".join(map(str, row)) for row in G) + "\n")
    write_text(tmp_path / "y.txt", "".join(map(str, y)) + "\n")
    print(f"case: program order {order} n={n} m={m} top_n={top_n}", flush=True)
    assert main([str(tmp_path / "g.txt"), str(tmp_path / "y.txt"), str(order), str(top_n),
                 str(tmp_path / "r.tsv")]) == 0
    ranks, snps, mi = parse_result(tmp_path / "r.tsv", order)
    r_or, m_or = oracle.scan(G, y, order, top_n)
    np.testing.assert_array_equal(ranks, r_or)
    np.testing.assert_array_equal(mi, m_or)
    for r, s in zip(ranks, snps):
        assert tuple(s) == oracle.unrank(n, order, int(r))
