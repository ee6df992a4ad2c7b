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


def _drawer(seed, scale=3.0):
    rng = np.random.default_rng(seed)
    return lambda k: [rng.normal(0.0, scale, 8) for _ in range(k)]


def test_elite_generation_keeps_one_in_ten_viable():
    """f_el is the lower 10 % quantile of the first batch of random genes,
    so 4 of 40 are viable there; the 5 elite genes all have fitness <= f_el
    and come in draw order; the same seed gives the same elite."""
    from paper_2306_15678_amd.ga import elite_generation
    calls = []

    def evaluate(pop):
        calls.append(len(pop))
        return _quadratic(pop)

    e = elite_generation(_drawer(1), evaluate, batch=40, size=5)
    first = _quadratic(_drawer(1)(40))
    assert e.f_el == float(np.sort(first)[3])
    assert int(np.sum(first <= e.f_el)) == 4
    assert len(e.genes) == 5 and np.all(e.losses <= e.f_el)
    assert np.array_equal(e.losses, _quadratic(e.genes))
    assert e.draws == 40 * len(calls) and len(calls) >= 2
    e2 = elite_generation(_drawer(1), _quadratic, batch=40, size=5)
    assert all(np.array_equal(a, b) for a, b in zip(e.genes, e2.genes))
    with pytest.raises(RuntimeError):
        elite_generation(_drawer(2), lambda pop: np.ones(len(pop)) * np.nan, batch=10,
                         size=5, max_batches=3)


def test_search_from_the_elite_generation():
    """The population starts with the elite genes and their children, and
    the search from there closes in on the minimum."""
    from paper_2306_15678_amd.ga import elite_generation
    e = elite_generation(_drawer(3), _quadratic, batch=40, size=5)
    cfg = GAConfig(population=10, generations=60, elite=2, mutation=0.3, floor=0.5, seed=5)
    s = GeneticSearch(np.zeros(8), cfg, elite=e)
    assert all(np.array_equal(a, b) for a, b in zip(s.pop[:5], e.genes)) and len(s.pop) == 10
    res = run(s, _quadratic, cfg.generations)
    assert res.best_loss < 0.05 * float(np.min(e.losses))
    with pytest.raises(ValueError):
        GeneticSearch(np.zeros(8), GAConfig(population=4), elite=e)


def test_degenerate_generation_is_replaced_by_the_elite():
    """Without carry-over elitism, an objective under which every child is
    far worse than its parents (fitness of anything not in the elite
    generation is large): each round the generation's best is worse than
    the elite gene, so the elite generation is reproduced in its place.
    With carry-over elitism the best never gets worse and it never is."""
    from paper_2306_15678_amd.ga import elite_generation
    e = elite_generation(_drawer(4), _quadratic, batch=40, size=5)
    keys = {g.tobytes() for g in e.genes}

    def hostile(pop):
        return np.array([_quadratic([x])[0] if x.tobytes() in keys else 1e6 for x in pop])

    cfg = GAConfig(population=8, generations=4, elite=0, seed=6)
    res = run(GeneticSearch(np.zeros(8), cfg, elite=e), hostile, cfg.generations)
    assert res.restorations == cfg.generations
    assert res.best_loss == float(np.min(e.losses))
    assert res.evaluations == cfg.population * (1 + 2 * cfg.generations)
    calm = run(GeneticSearch(np.zeros(8), GAConfig(population=8, generations=4, elite=1, seed=6),
                             elite=e), _quadratic, 4)
    assert calm.restorations == 0
