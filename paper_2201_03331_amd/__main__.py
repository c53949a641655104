"""The whole program of Fig. 1: read the variants, search, write the best
combinations.

    python -m paper_2201_03331_amd GENOTYPES PHENOTYPE ORDER TOP_N RESULT

Argument marshalling only: the files are read and written by the library's
I/O stage and the search runs on the GPU (fiuncho_scan).
"""
import argparse
import sys

from . import fiuncho


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2201_03331_amd", description=__doc__.splitlines()[0])
    ap.add_argument("genotypes", help="genotype file: one line of 0/1/2 per variant")
    ap.add_argument("phenotype", help="phenotype file: 0 (control) / 1 (case) per sample")
    ap.add_argument("order", type=int, help="interaction order k, 1..8")
    ap.add_argument("top_n", type=int, help="how many combinations to report")
    ap.add_argument("result", help="result file to write (tab-separated)")
    a = ap.parse_args(argv)
    G, y = fiuncho.read_dataset(a.genotypes, a.phenotype)
    hits = fiuncho.scan(G, y, a.order, a.top_n)
    fiuncho.write_hits(a.result, hits, a.order)
    print(f"{G.shape[0]} variants x {G.shape[1]} samples, order {a.order}: {len(hits)} combinations "
          f"written to {a.result}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
