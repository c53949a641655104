"""Seeded synthetic case/control genotype data.

The paper evaluates on datasets of 2048 samples per variant that it does not
describe further (section 5), so every workload here is generated.  This module
holds no part of the scan's arithmetic: it only draws inputs, which the tests,
the benchmark and the reference all consume.

Recipe
  * null variants: minor-allele frequency p ~ U[maf_lo, maf_hi]; genotype =
    number of minor alleles ~ Binomial(2, p) (Hardy-Weinberg), independent of
    the class;
  * planted interactions: a set S of variants with allele frequency 1/2, so
    genotype frequencies (1/4, 1/2, 1/4); per class, the joint genotype of S is
    drawn from P(g | case) ~ prod pi(g_i) f(g), P(g | control) ~ prod pi(g_i)
    (1 - f(g)) with penetrance f(g) = 1/2 + sum_sets delta * prod_{i in set}
    h(g_i), h = (+1, -1, +1).  Since E_pi[h] = 0, every proper subset of a set
    has no marginal effect: a pure interaction, the case exhaustive search is
    for (section 1);
  * m1 = round(case_fraction * m) cases, m - m1 controls, in shuffled order.
Genotypes are uint8 0/1/2 laid out [variant][sample]; the phenotype is uint8
0 (control) / 1 (case).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_PI = np.array([0.25, 0.5, 0.25])
_H = np.array([1.0, -1.0, 1.0])


@dataclass
class Dataset:
    genotypes: np.ndarray          # uint8 [n][m]
    phenotype: np.ndarray          # uint8 [m]
    order: int                     # interaction order to scan
    top_n: int
    planted: list = field(default_factory=list)   # list of sorted tuples
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.genotypes.shape[0])

    @property
    def m(self) -> int:
        return int(self.genotypes.shape[1])


def generate(n: int, m: int, *, seed: int, case_fraction: float = 0.5,
             maf: tuple = (0.05, 0.5), planted: list = (), order: int = 2,
             top_n: int = 10, name: str = "") -> Dataset:
    """Draw one dataset.  ``planted`` is a list of (size, delta) pairs; the
    sets are disjoint and their positions are drawn from the seed."""
    rng = np.random.default_rng(seed)
    m1 = int(round(case_fraction * m))
    m0 = m - m1
    y = np.concatenate([np.zeros(m0, np.uint8), np.ones(m1, np.uint8)])
    rng.shuffle(y)

    p = rng.uniform(maf[0], maf[1], size=n)
    G = rng.binomial(2, p[:, None], size=(n, m)).astype(np.uint8)

    sizes = [int(s) for s, _ in planted]
    total = sum(sizes)
    sets = []
    if total:
        pos = rng.choice(n, size=total, replace=False)
        at = 0
        for s in sizes:
            sets.append(tuple(sorted(int(v) for v in pos[at:at + s])))
            at += s
        # joint distribution over all planted variants (3**total cells)
        grids = np.indices((3,) * total).reshape(total, -1)          # [total][cells]
        prior = np.prod(_PI[grids], axis=0)
        f = np.full(grids.shape[1], 0.5)
        at = 0
        for (s, delta) in planted:
            f = f + float(delta) * np.prod(_H[grids[at:at + int(s)]], axis=0)
            at += int(s)
        assert np.all((f > 0) & (f < 1)), "penetrance out of (0,1)"
        for cls, w in ((1, prior * f), (0, prior * (1.0 - f))):
            idx = np.flatnonzero(y == cls)
            cells = rng.choice(grids.shape[1], size=idx.size, p=w / w.sum())
            # grid row r is the r-th drawn position (sets in draw order)
            for r in range(total):
                G[int(pos[r]), idx] = grids[r, cells].astype(np.uint8)
    return Dataset(G, y, order, top_n, sets, name)


# --- the workloads -----------------------------------------------------------

def order2_small() -> Dataset:
    """Order 2, 100 variants x 1,600 samples (800/800), one planted pair, top 10."""
    return generate(100, 1600, seed=1, planted=[(2, 0.2)], order=2, top_n=10,
                    name="order2-100x1600")


def order3_main() -> Dataset:
    """Order 3, 1,000 variants x 6,400 samples (balanced), one planted triple, top 100."""
    return generate(1000, 6400, seed=2, planted=[(3, 0.2)], order=3, top_n=100,
                    name="order3-1000x6400")


def order2_dense() -> Dataset:
    """Order 2, 4,000 variants x 16,000 samples (balanced), MAF U[0.01,0.5], top 1000."""
    return generate(4000, 16000, seed=3, maf=(0.01, 0.5), planted=[(2, 0.2)],
                    order=2, top_n=1000, name="order2-4000x16000")


def high_order(order: int) -> Dataset:
    """Orders 4/5, 200 variants x 4,000 samples, planted 4-way and 5-way sets, top 10."""
    return generate(200, 4000, seed=5, planted=[(4, 0.15), (5, 0.25)], order=order,
                    top_n=10, name=f"order{order}-200x4000")


def batch_jobs(count: int = 64, scale: float = 1.0) -> list:
    """64 uneven datasets: n ~ U{200..2000}, m ~ U{1000..20000}, case fraction
    ~ U[0.3,0.7], order 2 for even and 3 for odd job index, top 50 each.
    ``scale`` < 1 shrinks n and m (for quick tests) keeping the mix."""
    meta = np.random.default_rng(4)
    jobs = []
    for d in range(count):
        n = int(meta.integers(200, 2001))
        m = int(meta.integers(1000, 20001))
        frac = float(meta.uniform(0.3, 0.7))
        k = 2 if d % 2 == 0 else 3
        if scale != 1.0:
            n = max(k + 2, int(n * scale))
            m = max(8, int(m * scale))
        jobs.append(generate(n, m, seed=4000 + d, case_fraction=frac,
                             planted=[(k, 0.2)], order=k, top_n=50,
                             name=f"batch{d}-k{k}-{n}x{m}"))
    return jobs
