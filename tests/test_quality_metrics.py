"""The clustering scores of paper_1812_10048_amd.quality (host code, no GPU):
the Rand and adjusted Rand indices against scikit-learn's independent
implementations on random labelings, a hand-counted example, and the
invariances (relabelling, identical partitions)."""
import numpy as np
from sklearn.metrics import adjusted_rand_score, rand_score

from paper_1812_10048_amd import quality


def test_scores_match_scikit_learn_on_random_labelings():
    rng = np.random.default_rng(0)
    for n, ka, kb in [(10, 2, 3), (200, 5, 5), (5000, 12, 40), (3, 1, 3)]:
        a = rng.integers(0, ka, size=n)
        b = rng.integers(0, kb, size=n)
        assert abs(quality.adjusted_rand_index(a, b) - adjusted_rand_score(a, b)) < 1e-12
        assert abs(quality.rand_index(a, b) - rand_score(a, b)) < 1e-12
        assert abs(quality.hubert_index(a, b) - (2 * rand_score(a, b) - 1)) < 1e-12


def test_hand_counted_example_and_invariances():
    a = np.array([0, 0, 1, 1])
    b = np.array([0, 1, 0, 1])
    # pairs: together in a (0,1),(2,3); in b (0,2),(1,3); apart in both (0,3),(1,2)
    assert abs(quality.rand_index(a, b) - 2 / 6) < 1e-15
    assert abs(quality.hubert_index(a, b) - (-1 / 3)) < 1e-15
    rng = np.random.default_rng(1)
    z = rng.integers(0, 6, size=500)
    perm = rng.permutation(6)
    assert quality.adjusted_rand_index(z, perm[z] + 100) == 1.0
    assert quality.rand_index(z, z) == 1.0


def test_recipe_variants_change_only_the_named_field():
    import dataclasses

    from paper_1812_10048_amd import synth
    from paper_1812_10048_amd.quality import recipe_variant

    base = synth.RECIPES["c2"]
    r = recipe_variant("c2", lib_mean=250)
    assert (r.lib_mean, r.conc, r.n_cells, r.sizes) == (250.0, base.conc, base.n_cells, base.sizes)
    assert r.name == "c2-lib250"
    r = recipe_variant("c2", conc=0.5)
    assert (r.lib_mean, r.conc, r.name) == (base.lib_mean, 0.5, "c2-conc0.5")
    assert recipe_variant("c1") == synth.RECIPES["c1"]
    # a shallower library gives sparser rows at the same seed
    small = synth.generate(dataclasses.replace(synth.RECIPES["c1"], lib_mean=100.0), seed=0, n_cells=300)
    deep = synth.generate(synth.RECIPES["c1"], seed=0, n_cells=300)
    assert small.nnz < deep.nnz
