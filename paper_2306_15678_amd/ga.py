"""Genetic-algorithm search for the screen parameters (the paper's optimiser).

The paper fits its effective-lens parameters with a classical genetic
algorithm whose fitness is the mismatch between the sparse-grid solution and
a dense-grid reference (Math and Equations: gene vector D, penalty from the
solution difference).  Here the genes are the 8 ansatz parameters theta.
The whole population marches as one batch on the GPU (one instance per
individual, so every pass is one launch for all of them) and the fitness is
the library's fluence mismatch against the target.

Operators (one seeded generator drives all of them): the best `elite`
individuals pass unchanged; parents are drawn with probability
proportional to 1/loss (roulette); a child is a random convex blend of two
parents gene by gene, then a Gaussian mutation of relative size `mutation`
(with an absolute floor).  With elitism the best loss never increases.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from .march import Propagator


@dataclass
class GAConfig:
    population: int = 8
    generations: int = 10
    elite: int = 1
    mutation: float = 0.1   # std of the mutation relative to max(|gene|, floor)
    floor: float = 0.1
    seed: int = 0


@dataclass
class GAResult:
    best: np.ndarray
    best_loss: float
    history: List[float] = field(default_factory=list)  # best loss of each generation
    evaluations: int = 0


class GeneticSearch:
    """Population bookkeeping and operators, independent of the evaluator."""

    def __init__(self, start: Sequence[float], cfg: GAConfig):
        if cfg.population < 2 or not (0 <= cfg.elite < cfg.population):
            raise ValueError("need population >= 2 and 0 <= elite < population")
        self.cfg = cfg
        self.rng = np.random.default_rng(cfg.seed)
        x0 = np.asarray(start, dtype=np.float64)
        # the start and population - 1 mutants of it
        self.pop = [x0.copy()] + [self._mutate(x0) for _ in range(cfg.population - 1)]

    def _mutate(self, x: np.ndarray) -> np.ndarray:
        scale = self.cfg.mutation * np.maximum(np.abs(x), self.cfg.floor)
        return x + self.rng.normal(0.0, 1.0, x.shape) * scale

    def next_generation(self, loss: np.ndarray) -> List[np.ndarray]:
        loss = np.asarray(loss, dtype=np.float64)
        order = np.argsort(loss, kind="stable")
        new = [self.pop[i].copy() for i in order[:self.cfg.elite]]
        fit = 1.0 / np.maximum(loss, 1e-300)
        prob = fit / fit.sum()
        while len(new) < self.cfg.population:
            a, b = self.rng.choice(len(self.pop), size=2, p=prob)
            w = self.rng.random(self.pop[a].shape)
            new.append(self._mutate(w * self.pop[a] + (1.0 - w) * self.pop[b]))
        self.pop = new
        return self.pop


def run(search: GeneticSearch, evaluate: Callable[[List[np.ndarray]], np.ndarray],
        generations: int) -> GAResult:
    """Evaluate the population, then `generations` rounds of selection,
    crossover, mutation and evaluation."""
    loss = np.asarray(evaluate(search.pop), dtype=np.float64)
    res = GAResult(best=search.pop[int(np.argmin(loss))].copy(), best_loss=float(loss.min()),
                   history=[float(loss.min())], evaluations=len(loss))
    for _ in range(generations):
        pop = search.next_generation(loss)
        loss = np.asarray(evaluate(pop), dtype=np.float64)
        res.evaluations += len(loss)
        k = int(np.argmin(loss))
        if loss[k] < res.best_loss:
            res.best, res.best_loss = pop[k].copy(), float(loss[k])
        res.history.append(float(loss.min()))
    return res


def population_evaluator(prop: Propagator, u0, target, n_steps: int):
    """Fitness of a list of theta vectors: every individual is one instance
    of `prop` (all on the same grid), marched together from u0."""
    dev = prop.device
    u0_d = torch.as_tensor(u0).to(dev)
    t_d = torch.as_tensor(target, dtype=torch.float64).to(dev)

    def evaluate(pop: List[np.ndarray]) -> np.ndarray:
        if len(pop) != prop.n_inst:
            raise ValueError("population size must equal the context's instance count")
        for b, th in enumerate(pop):
            prop.set_field(b, u0_d)
            prop.set_theta(b, th)
        prop.propagate(n_steps)
        return np.array([prop.fluence_mismatch(b, t_d) for b in range(len(pop))])

    return evaluate


def fit_theta(desc, u0, target, theta0: Sequence[float], n_steps: int,
              cfg: Optional[GAConfig] = None, precision: int = 32) -> GAResult:
    """GA fit of the ansatz parameters of one beam (descriptor `desc`) to a
    target fluence after n_steps, the population batched in one context."""
    cfg = cfg or GAConfig()
    prop = Propagator([desc] * cfg.population, precision=precision)
    try:
        search = GeneticSearch(theta0, cfg)
        return run(search, population_evaluator(prop, u0, target, n_steps), cfg.generations)
    finally:
        prop.close()
