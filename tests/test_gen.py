"""Seeded generators: determinism and the shape of each workload (CPU)."""
import numpy as np

from paper_0811_3301_amd import gen


def test_random_walk_definition_and_seed():
    a = gen.random_walk(5, 64, gen.rng(2, 0))
    b = gen.random_walk(5, 64, gen.rng(2, 0))
    assert np.array_equal(a, b)
    assert np.all(a[:, 0] == 0.0)
    steps = np.diff(gen.random_walk(2000, 64, gen.rng(9, 0)), axis=1)
    assert abs(steps.mean()) < 0.01 and abs(steps.std() - 1.0) < 0.01


def test_queries_are_fresh_draws():
    db, qs = gen.make_workload("rw128_small")
    assert db.shape == (1000, 128) and qs.shape == (16, 128)
    assert not any(np.array_equal(q, d) for q in qs for d in db[:50])


def test_shape_signatures_are_znormalised():
    s = gen.shape_signatures(20, 512, gen.rng(3, 0))
    assert s.shape == (20, 512)
    assert np.allclose(s.mean(axis=1), 0.0, atol=1e-9)
    assert np.allclose(s.std(axis=1), 1.0, atol=1e-9)
    # smooth: neighbouring samples are strongly correlated
    assert np.mean(np.abs(np.diff(s, axis=1))) < 0.2


def test_band_fractions():
    assert [gen.band_from_fraction(n, 0.1) for n in (128, 256, 512)] == [13, 26, 51]
    assert [gen.band_from_fraction(1024, f) for f in (0.05, 0.1, 0.2)] == [51, 102, 205]
    assert gen.band_from_fraction(64, 0.05) == 3


def test_poisson_arrivals():
    t = gen.poisson_arrivals(1000.0, 20000, gen.rng(5, 2))
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1e-3) < 3e-5
