"""Genetic-search operators on a cheap objective (no GPU): elitism keeps the
best loss non-increasing, the search closes in on a known minimum, and a
seed fixes the whole run."""
import numpy as np
import pytest

from paper_2306_15678_amd.ga import GAConfig, GeneticSearch, run

X_STAR = np.array([0.3, -1.2, 2.0, 0.5, -0.7, 1.1, 0.0, -2.5])


def _quadratic(pop):
    return np.array([1e-3 + float(np.sum((x - X_STAR) ** 2)) for x in pop])


def test_search_improves_and_keeps_the_best():
    cfg = GAConfig(population=16, generations=60, elite=2, mutation=0.3, floor=0.5, seed=4)
    res = run(GeneticSearch(np.zeros(8), cfg), _quadratic, cfg.generations)
    assert all(b <= a for a, b in zip(res.history, res.history[1:]))
    assert res.best_loss < 0.05 * _quadratic([np.zeros(8)])[0]
    assert res.best_loss == pytest.approx(_quadratic([res.best])[0], rel=0, abs=0)
    assert res.evaluations == cfg.population * (cfg.generations + 1)


def test_seed_fixes_the_run():
    cfg = GAConfig(population=8, generations=10, seed=11)
    a = run(GeneticSearch(np.ones(8), cfg), _quadratic, cfg.generations)
    b = run(GeneticSearch(np.ones(8), cfg), _quadratic, cfg.generations)
    assert a.history == b.history and np.array_equal(a.best, b.best)
    c = run(GeneticSearch(np.ones(8), GAConfig(population=8, generations=10, seed=12)),
            _quadratic, 10)
    assert c.history != a.history


def test_start_is_in_the_first_population_and_bad_configs_fail():
    s = GeneticSearch(np.arange(8.0), GAConfig(population=5))
    assert np.array_equal(s.pop[0], np.arange(8.0)) and len(s.pop) == 5
    with pytest.raises(ValueError):
        GeneticSearch(np.zeros(8), GAConfig(population=1))
    with pytest.raises(ValueError):
        GeneticSearch(np.zeros(8), GAConfig(population=4, elite=4))
