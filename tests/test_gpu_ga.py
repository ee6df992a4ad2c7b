"""The genetic search on the GPU: population fitness from one batched march.

Fitness values are checked against each individual marched alone (bitwise)
and against the FP64 oracle's loss; the search itself by its invariants
(non-increasing best loss, the reported best re-evaluates to its loss, a
seed fixes the run) on a twin target whose parameters are known.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import march as M
from paper_2306_15678_amd.ga import GAConfig, GeneticSearch, fit_theta, population_evaluator, run
from paper_2306_15678_amd.march import Propagator, desc_of

pytestmark = pytest.mark.gpu

STEPS = 100  # config 4 sparse before its collapse (about step 150)


def _twin():
    inst = W.config4_sparse()
    u0 = W.initial_field(inst)
    theta_true = np.array(inst.theta) + W.random_theta(8, 0.05)
    p = Propagator([desc_of(inst)], precision=64)
    p.set_field(0, u0)
    p.set_theta(0, theta_true)
    p.propagate(STEPS)
    target = p.intensity(0)
    p.close()
    return inst, u0, theta_true, target


def _population(inst, k, seed):
    rng = np.random.default_rng(seed)
    return [np.array(inst.theta) + 0.1 * rng.standard_normal(8) for _ in range(k)]


@pytest.mark.parametrize("precision", [32, 64])
def test_batched_fitness_equals_each_individual_alone(precision):
    inst, u0, _, target = _twin()
    pop = _population(inst, 4, 1)
    p = Propagator([desc_of(inst)] * 4, precision=precision)
    batched = population_evaluator(p, u0, target, STEPS)(pop)
    p.close()
    for b, th in enumerate(pop):
        q = Propagator([desc_of(inst)], precision=precision)
        alone = population_evaluator(q, u0, target, STEPS)([th])[0]
        q.close()
        assert alone == batched[b]


def test_fp64_fitness_matches_the_oracle():
    inst, u0, _, target = _twin()
    pop = _population(inst, 3, 2)
    p = Propagator([desc_of(inst)] * 3, precision=64)
    got = population_evaluator(p, u0, target, STEPS)(pop)
    p.close()
    for th, g in zip(pop, got):
        r = M.march(u0, inst, n_steps=STEPS, theta=th)
        want = M.fluence_loss(r.field, target)[0]
        assert abs(g / want - 1) < 1e-11, (g, want)


def test_search_on_a_twin_target():
    inst, u0, theta_true, target = _twin()
    cfg = GAConfig(population=8, generations=6, elite=1, mutation=0.05, floor=0.05, seed=3)
    res = fit_theta(desc_of(inst), u0, target, inst.theta, STEPS, cfg, precision=32)
    assert all(b <= a for a, b in zip(res.history, res.history[1:]))
    q = Propagator([desc_of(inst)], precision=32)
    ev = population_evaluator(q, u0, target, STEPS)
    start = ev([np.array(inst.theta)])[0]
    assert res.best_loss <= start and ev([res.best])[0] == res.best_loss
    q.close()
    again = fit_theta(desc_of(inst), u0, target, inst.theta, STEPS, cfg, precision=32)
    assert again.history == res.history
    print(f"GA twin: loss at theta0 {start:.3e} -> best {res.best_loss:.3e} after "
          f"{res.evaluations} marches; |theta - theta_true| {np.linalg.norm(res.best - theta_true):.3e} "
          f"(from {np.linalg.norm(np.array(inst.theta) - theta_true):.3e})", flush=True)


def test_mismatch_leaves_the_recorded_adjoint_alone():
    inst, u0, _, target = _twin()
    other = W.synthetic_target(inst, 7)
    grads = []
    for with_mismatch in (False, True):
        p = Propagator([desc_of(inst)], precision=32, max_steps=STEPS, ckpt_every=25)
        p.set_field(0, u0)
        p.set_theta(0, np.array(inst.theta))
        p.forward_record(STEPS)
        loss = p.fluence_loss(0, target)
        if with_mismatch:
            assert p.fluence_mismatch(0, target) == loss
            p.fluence_mismatch(0, other)
        p.backward()
        grads.append((p.grad_theta(0), p.grad_field(0)))
        p.close()
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])


# --------------------------------------------- measure-vector fitness
def _p0(inst, u0, theta, w_p):
    """P0 of the twin march, from the oracle's FP64 fluence."""
    from oracle import diagnostics as D
    r = M.march(u0, inst, n_steps=STEPS, theta=theta)
    w = np.abs(r.field) ** 2
    return D.measure_vector(w, inst.length, w_p), w


def test_measure_vector_and_distance_match_the_oracle():
    """The library's measure vector of the FP64 march's fluence and its
    distance from the twin's P0 against the oracle's (moments and peak to
    FP64 summation order, the hot-area count exactly); batched distances
    equal each individual alone bitwise (FP32 and FP64)."""
    from oracle import diagnostics as D
    inst, u0, theta_true, _ = _twin()
    w_p = 0.05 * W.I_A
    p0, w_true = _p0(inst, u0, theta_true, w_p)
    assert p0[5] >= 1
    pop = _population(inst, 3, 5)
    p = Propagator([desc_of(inst)] * 3, precision=64)
    got = p.measure_vector(torch.from_numpy(w_true).cuda(), inst.length, w_p)
    assert np.max(np.abs(got[:5] / p0[:5] - 1)) < 1e-12 and got[5] == p0[5]
    dist = population_evaluator(p, u0, None, STEPS, fitness="measure", p0=p0, w_p=w_p)(pop)
    for b, th in enumerate(pop):
        r = M.march(u0, inst, n_steps=STEPS, theta=th)
        want_p = D.measure_vector(np.abs(r.field) ** 2, inst.length, w_p)
        want = D.measure_distance(want_p, p0)
        d, pv = p.measure_distance(b, p0, w_p)
        print(f"measure distance {b}: {d:.6e} (oracle {want:.6e})", flush=True)
        assert pv[5] == want_p[5]
        assert np.max(np.abs(pv[:5] / want_p[:5] - 1)) < 1e-11
        assert abs(dist[b] / want - 1) < 1e-11 and dist[b] == d
    p.close()
    for precision in (32, 64):
        q = Propagator([desc_of(inst)] * 3, precision=precision)
        batched = population_evaluator(q, u0, None, STEPS, fitness="measure", p0=p0, w_p=w_p)(pop)
        q.close()
        for b, th in enumerate(pop):
            s = Propagator([desc_of(inst)], precision=precision)
            alone = population_evaluator(s, u0, None, STEPS, fitness="measure", p0=p0,
                                         w_p=w_p)([th])[0]
            s.close()
            assert alone == batched[b]


def test_elite_generation_and_search_on_the_measure_fitness():
    """The paper's procedure on the GPU: random genes around theta0 in
    batches of the population size, an elite generation of 5 with f_el the
    10 % quantile, then the search from it on the measure distance to the
    twin's P0 without carry-over elitism (the elite generation is restored
    when a generation's best falls behind the elite gene); the best
    distance never exceeds the elite's best."""
    from paper_2306_15678_amd.ga import elite_generation
    inst, u0, theta_true, _ = _twin()
    w_p = 0.05 * W.I_A
    p0, _ = _p0(inst, u0, theta_true, w_p)
    cfg = GAConfig(population=10, generations=5, elite=0, mutation=0.05, floor=0.1, seed=3)
    p = Propagator([desc_of(inst)] * cfg.population, precision=32)
    ev = population_evaluator(p, u0, None, STEPS, fitness="measure", p0=p0, w_p=w_p)
    rng = np.random.default_rng(9)
    draw = lambda k: [np.array(inst.theta) + 0.1 * rng.standard_normal(8) for _ in range(k)]
    e = elite_generation(draw, ev, batch=cfg.population, size=5)
    assert len(e.genes) == 5 and np.all(e.losses <= e.f_el)
    res = run(GeneticSearch(inst.theta, cfg, elite=e), ev, cfg.generations)
    print(f"elite f_el {e.f_el:.4e} best {e.losses.min():.4e} -> GA {res.best_loss:.4e}, "
          f"restorations {res.restorations}", flush=True)
    assert res.best_loss <= float(e.losses.min())
    p.close()
