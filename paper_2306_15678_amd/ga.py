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

The paper's start (GA paragraph, Fig. 2): a first viable ("elite")
generation of 5 is picked from random genes, keeping those whose fitness is
below a level f_el chosen so that about one random gene in 10 is viable;
when a generation ends up worse than the elite gene, its degenerate
descendants are discarded and the elite generation is reproduced again.  Fitness is either the fluence mismatch against a target
or the distance of the solution's measure vector P from the dense-grid
P0 (Euclidean, in relative units; ssfm_measure_distance).
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
    restorations: int = 0       # generations replaced by the elite generation


@dataclass
class EliteSet:
    """The first viable generation: genes with fitness <= f_el."""
    genes: List[np.ndarray]
    losses: np.ndarray
    f_el: float
    draws: int                  # random genes evaluated to find them


def elite_generation(draw: Callable[[int], List[np.ndarray]],
                     evaluate: Callable[[List[np.ndarray]], np.ndarray], batch: int,
                     size: int = 5, viable: float = 0.1, max_batches: int = 100) -> EliteSet:
    """Random genes in batches of `batch` (one batched evaluation each): f_el
    is the `viable` quantile of the first batch's fitness (the lower sample,
    so that about that fraction of random genes qualifies), then genes with
    fitness <= f_el are kept, in draw order, until `size` are found."""
    if batch < 1 or size < 1 or not (0.0 < viable < 1.0):
        raise ValueError("need batch >= 1, size >= 1, 0 < viable < 1")
    genes: List[np.ndarray] = []
    losses: List[float] = []
    f_el = None
    draws = 0
    for _ in range(max_batches):
        cand = draw(batch)
        loss = np.asarray(evaluate(cand), dtype=np.float64)
        draws += len(cand)
        if f_el is None:
            f_el = float(np.quantile(loss, viable, method="lower"))
        for x, l in zip(cand, loss):
            if l <= f_el and len(genes) < size:
                genes.append(np.asarray(x, dtype=np.float64).copy())
                losses.append(float(l))
        if len(genes) >= size:
            return EliteSet(genes, np.array(losses), f_el, draws)
    raise RuntimeError(f"only {len(genes)} viable genes in {draws} draws (f_el = {f_el})")


class GeneticSearch:
    """Population bookkeeping and operators, independent of the evaluator."""

    def __init__(self, start: Sequence[float], cfg: GAConfig,
                 elite: Optional[EliteSet] = None):
        if cfg.population < 2 or not (0 <= cfg.elite < cfg.population):
            raise ValueError("need population >= 2 and 0 <= elite < population")
        self.cfg = cfg
        self.rng = np.random.default_rng(cfg.seed)
        self.elite_set = elite
        if elite is not None:
            if len(elite.genes) > cfg.population:
                raise ValueError("the elite generation is larger than the population")
            self.pop = self.from_elite()
        else:
            x0 = np.asarray(start, dtype=np.float64)
            # the start and population - 1 mutants of it
            self.pop = [x0.copy()] + [self._mutate(x0) for _ in range(cfg.population - 1)]

    def _mutate(self, x: np.ndarray) -> np.ndarray:
        scale = self.cfg.mutation * np.maximum(np.abs(x), self.cfg.floor)
        return x + self.rng.normal(0.0, 1.0, x.shape) * scale

    def _breed(self, parents: List[np.ndarray], prob: np.ndarray) -> np.ndarray:
        a, b = self.rng.choice(len(parents), size=2, p=prob)
        w = self.rng.random(parents[a].shape)
        return self._mutate(w * parents[a] + (1.0 - w) * parents[b])

    @staticmethod
    def _roulette(loss: np.ndarray) -> np.ndarray:
        fit = 1.0 / np.maximum(np.asarray(loss, dtype=np.float64), 1e-300)
        return fit / fit.sum()

    def from_elite(self) -> List[np.ndarray]:
        """The elite generation reproduced: its genes, then children of them
        (roulette on their fitness) up to the population size."""
        e = self.elite_set
        pop = [g.copy() for g in e.genes]
        prob = self._roulette(e.losses)
        while len(pop) < self.cfg.population:
            pop.append(self._breed(e.genes, prob))
        return pop

    def next_generation(self, loss: np.ndarray) -> List[np.ndarray]:
        loss = np.asarray(loss, dtype=np.float64)
        order = np.argsort(loss, kind="stable")
        new = [self.pop[i].copy() for i in order[:self.cfg.elite]]
        prob = self._roulette(loss)
        while len(new) < self.cfg.population:
            new.append(self._breed(self.pop, prob))
        self.pop = new
        return self.pop


def run(search: GeneticSearch, evaluate: Callable[[List[np.ndarray]], np.ndarray],
        generations: int) -> GAResult:
    """Evaluate the population, then `generations` rounds of selection,
    crossover, mutation and evaluation.  With an elite generation, a
    generation whose best fitness is worse than the elite gene's (the best
    of the elite generation) is discarded and the elite generation
    reproduced in its place (and evaluated) before the next round; with
    carry-over elitism (cfg.elite >= 1) the best never gets worse, so this
    acts only when carry-over is off."""
    loss = np.asarray(evaluate(search.pop), dtype=np.float64)
    res = GAResult(best=search.pop[int(np.argmin(loss))].copy(), best_loss=float(loss.min()),
                   history=[float(loss.min())], evaluations=len(loss))
    elite = search.elite_set
    for _ in range(generations):
        pop = search.next_generation(loss)
        loss = np.asarray(evaluate(pop), dtype=np.float64)
        res.evaluations += len(loss)
        k = int(np.argmin(loss))
        if loss[k] < res.best_loss:
            res.best, res.best_loss = pop[k].copy(), float(loss[k])
        res.history.append(float(loss.min()))
        if elite is not None and float(loss.min()) > float(elite.losses.min()):
            search.pop = search.from_elite()
            loss = np.asarray(evaluate(search.pop), dtype=np.float64)
            res.evaluations += len(loss)
            res.restorations += 1
    return res


def population_evaluator(prop: Propagator, u0, target, n_steps: int,
                         fitness: str = "mismatch", p0: Optional[Sequence[float]] = None,
                         w_p: Optional[float] = None):
    """Fitness of a list of theta vectors: every individual is one instance
    of `prop` (all on the same grid), marched together from u0.  fitness
    "mismatch": the fluence mismatch against `target`; "measure": the
    distance of the measure vector P of each fluence from p0 (hot areas at
    w_p; target unused)."""
    if fitness not in ("mismatch", "measure"):
        raise ValueError("fitness is 'mismatch' or 'measure'")
    if fitness == "measure" and (p0 is None or w_p is None):
        raise ValueError("the measure fitness needs p0 and w_p")
    dev = prop.device
    u0_d = torch.as_tensor(u0).to(dev)
    t_d = torch.as_tensor(target, dtype=torch.float64).to(dev) if fitness == "mismatch" else None

    def evaluate(pop: List[np.ndarray]) -> np.ndarray:
        if len(pop) != prop.n_inst:
            raise ValueError("population size must equal the context's instance count")
        for b, th in enumerate(pop):
            prop.set_field(b, u0_d)
            prop.set_theta(b, th)
        prop.propagate(n_steps)
        if fitness == "measure":
            return np.array([prop.measure_distance(b, p0, w_p)[0] for b in range(len(pop))])
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
