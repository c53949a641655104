"""The seeded generator draws what its recipe says (no method arithmetic here)."""
import numpy as np

from paper_2201_03331_amd import synth


def test_shapes_classes_and_determinism():
    d = synth.generate(50, 1001, seed=9, case_fraction=0.3, planted=[(2, 0.2)], order=2)
    assert d.genotypes.shape == (50, 1001) and d.genotypes.dtype == np.uint8
    assert d.phenotype.shape == (1001,) and set(np.unique(d.phenotype)) <= {0, 1}
    assert int(d.phenotype.sum()) == round(0.3 * 1001)
    assert d.genotypes.max() <= 2
    # classes are interleaved, not blocked
    assert 0 < np.flatnonzero(d.phenotype)[0] < 1001 - 300
    d2 = synth.generate(50, 1001, seed=9, case_fraction=0.3, planted=[(2, 0.2)], order=2)
    np.testing.assert_array_equal(d.genotypes, d2.genotypes)
    np.testing.assert_array_equal(d.phenotype, d2.phenotype)


def test_hardy_weinberg_and_maf():
    d = synth.generate(400, 20000, seed=3, maf=(0.05, 0.5))
    G = d.genotypes.astype(np.float64)
    p = G.mean(axis=1) / 2.0
    assert p.min() > 0.03 and p.max() < 0.52
    # heterozygote frequency close to 2p(1-p)
    het = (d.genotypes == 1).mean(axis=1)
    assert np.abs(het - 2 * p * (1 - p)).max() < 0.02


def test_planted_sets_have_no_marginal_effect_but_joint_effect():
    d = synth.generate(20, 60000, seed=4, planted=[(3, 0.2)], order=3)
    (a, b, c) = d.planted[0]
    y = d.phenotype
    for v in (a, b, c):
        for g in range(3):
            sel = d.genotypes[v] == g
            assert abs(y[sel].mean() - y.mean()) < 0.02
    par = ((d.genotypes[a] == 1).astype(int) + (d.genotypes[b] == 1) + (d.genotypes[c] == 1)) % 2
    # odd number of heterozygotes -> penetrance 0.3, even -> 0.7
    assert y[par == 0].mean() > 0.6 and y[par == 1].mean() < 0.4


def test_workload_shapes():
    d = synth.order2_small()
    assert (d.n, d.m, d.order, d.top_n) == (100, 1600, 2, 10)
    assert int(d.phenotype.sum()) == 800
    jobs = synth.batch_jobs(8, scale=0.05)
    assert [j.order for j in jobs] == [2, 3] * 4
