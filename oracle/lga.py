"""Lamarckian genetic algorithm with ADADELTA local search (oracle).

What the paper fixes (Background, "Design and Structure of MiniMDock"): a
population of candidate poses is evolved by crossover and fitness-based
selection; each generation a local optimisation is applied to a random sample of
individuals and its result is written back into the population (Lamarckian);
several independent runs, each starting from 150 individuals, proceed at once and
the answer is the best pose over all runs.  Evaluations are counted per
individual and summed per run (Section "Removing architecture-specific code",
the sum_evals listings), which drives termination.

Operator choices (readings; the paper names the operators only -- parity
unpinned beyond the invariants, the small-ligand lattice minima and the sampler's
distribution that the tests check):
  * initial individual: translation uniform in the grid box, orientation a uniform
    random unit quaternion (Shoemake's method from three uniforms), torsions
    uniform in (-pi, pi];
  * elitism 1: the best individual (lowest energy, ties to the lower index) is
    copied unchanged into slot 0 without a new evaluation;
  * every other slot: two parents, each the winner of a binary tournament (two
    uniform picks, the better one wins with probability tournament_rate);
    two-point crossover with probability crossover_rate over the gene units
    [t_x, t_y, t_z, q, theta_1 .. theta_T] (the quaternion is one unit), the child
    taking parent B's units in [lo, hi) and parent A's elsewhere; then per unit,
    with probability mutation_rate, t += U(-2, 2) A, q <- normalise(r (x) q) for r a
    rotation by U(-pi/2, pi/2) about a uniform random axis, theta += U(-pi, pi)
    wrapped to (-pi, pi];
  * local search on ceil(ls_rate * pop) distinct individuals: those whose random
    key (ties to the lower index) ranks lowest;
  * local optimiser: ADADELTA (`adadelta`, the default) or Solis-Wets (`solis_wets`,
    ls_method="solis_wets"), which the paper names; either spends exactly ls_iters
    evaluations per searched individual;
  * evaluation budget: each GA evaluation counts 1, each local-search evaluation 1; the
    budget is checked at generation boundaries (the last generation may overshoot).
Random numbers: `rng` (a counter-based draw per decision).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import rng as R
from .adadelta import local_search
from .solis_wets import local_search_sw
from .pose import quat_mul, wrap_angle
from .scoring import energy


@dataclass
class DockParams:
    n_runs: int = 1
    pop_size: int = 150
    max_generations: int = 10
    max_evals_per_run: int = 10 ** 12
    ls_rate: float = 0.06
    ls_iters: int = 300
    rho: float = 0.8
    eps: float = 1e-2
    crossover_rate: float = 0.8
    mutation_rate: float = 0.02
    tournament_rate: float = 0.6
    elitism: int = 1
    mut_trans: float = 2.0
    mut_rot: float = math.pi / 2
    mut_tors: float = math.pi
    seed: int = 7
    ls_method: str = "adadelta"


def n_local_search(p: DockParams) -> int:
    """ceil(ls_rate * pop_size), tolerant of the rate's binary rounding."""
    return max(0, min(p.pop_size, int(math.ceil(p.ls_rate * p.pop_size - 1e-4))))


def evals_per_generation(p: DockParams) -> int:
    return (p.pop_size - p.elitism) + n_local_search(p) * p.ls_iters


def planned_generations(p: DockParams) -> int:
    """Generations run: stop at the first boundary where the budget is reached."""
    evals, gens = p.pop_size, 0
    per = evals_per_generation(p)
    while gens < p.max_generations and evals < p.max_evals_per_run:
        gens += 1
        evals += per
    return gens


def initial_individual(grid, lig, p: DockParams, run: int, indiv: int) -> np.ndarray:
    G = lig.n_genes
    x = np.zeros(G)
    lo = grid.origin
    hi = grid.origin + (grid.n_xyz - 1) * grid.spacing

    def u(idx):
        return R.uniform(p.seed, run, 0, indiv, R.P_INIT, idx)

    for a in range(3):
        x[a] = lo[a] + u(a) * (hi[a] - lo[a])
    u1, u2, u3 = u(3), u(4), u(5)
    s1, s2 = math.sqrt(1.0 - u1), math.sqrt(u1)
    x[3] = s1 * math.sin(2.0 * math.pi * u2)
    x[4] = s1 * math.cos(2.0 * math.pi * u2)
    x[5] = s2 * math.sin(2.0 * math.pi * u3)
    x[6] = s2 * math.cos(2.0 * math.pi * u3)
    for k in range(lig.n_torsions):
        x[7 + k] = math.pi - 2.0 * math.pi * u(6 + k)
    return x


def _better(E, a, b):
    return a if (E[a] < E[b] or (E[a] == E[b] and a <= b)) else b


def tournament(E, p: DockParams, run, gen, slot, which):
    base = 3 * which
    a = R.randint(p.pop_size, p.seed, run, gen, slot, R.P_TOURNAMENT, base)
    b = R.randint(p.pop_size, p.seed, run, gen, slot, R.P_TOURNAMENT, base + 1)
    u = R.uniform(p.seed, run, gen, slot, R.P_TOURNAMENT, base + 2)
    best = _better(E, a, b)
    worst = b if best == a else a
    return best if u < p.tournament_rate else worst


def _units(lig):
    return 4 + lig.n_torsions


def crossover(xa, xb, lig, p: DockParams, run, gen, slot):
    child = xa.copy()
    if R.uniform(p.seed, run, gen, slot, R.P_CROSSOVER, 0) < p.crossover_rate:
        U = _units(lig)
        c1 = R.randint(U + 1, p.seed, run, gen, slot, R.P_CROSSOVER, 1)
        c2 = R.randint(U + 1, p.seed, run, gen, slot, R.P_CROSSOVER, 2)
        lo, hi = min(c1, c2), max(c1, c2)
        for m in range(lo, hi):
            if m < 3:
                child[m] = xb[m]
            elif m == 3:
                child[3:7] = xb[3:7]
            else:
                child[7 + m - 4] = xb[7 + m - 4]
    return child


def mutate(x, lig, p: DockParams, run, gen, slot):
    x = x.copy()

    def u(idx):
        return R.uniform(p.seed, run, gen, slot, R.P_MUTATION, idx)

    for m in range(_units(lig)):
        if u(4 * m) >= p.mutation_rate:
            continue
        if m < 3:
            x[m] += (2.0 * u(4 * m + 1) - 1.0) * p.mut_trans
        elif m == 3:
            alpha = (2.0 * u(4 * m + 1) - 1.0) * p.mut_rot
            z = 2.0 * u(4 * m + 2) - 1.0
            phi = 2.0 * math.pi * u(4 * m + 3)
            rxy = math.sqrt(max(0.0, 1.0 - z * z))
            axis = np.array([rxy * math.cos(phi), rxy * math.sin(phi), z])
            r = np.concatenate([[math.cos(0.5 * alpha)], math.sin(0.5 * alpha) * axis])
            qn = quat_mul(r, x[3:7])
            x[3:7] = qn / np.linalg.norm(qn)
        else:
            k = m - 4
            x[7 + k] = wrap_angle(x[7 + k] + (2.0 * u(4 * m + 1) - 1.0) * p.mut_tors)
    return x


def local_search_picks(p: DockParams, run, gen):
    """Indices chosen for local search, in rank order of their random keys."""
    keys = [R.draw_u24(p.seed, run, gen, i, R.P_LS_PICK, 0) for i in range(p.pop_size)]
    order = sorted(range(p.pop_size), key=lambda i: (keys[i], i))
    return order[:n_local_search(p)]


def argbest(E):
    """Index of the lowest energy, ties to the lower index."""
    b = 0
    for i in range(1, len(E)):
        if E[i] < E[b]:
            b = i
    return b


def run_lga(grid, lig, p: DockParams, run: int, trace=None):
    """One independent run.  Returns (best_genes, best_energy, evals, generations)."""
    pop = [initial_individual(grid, lig, p, run, i) for i in range(p.pop_size)]
    E = [energy(grid, lig, x) for x in pop]
    evals = p.pop_size
    if trace is not None:
        trace.append(dict(gen=0, genes=np.array(pop), energy=np.array(E), evals=evals))
    gen = 0
    n_ls = n_local_search(p)
    while gen < p.max_generations and evals < p.max_evals_per_run:
        gen += 1
        new, newE = [None] * p.pop_size, [None] * p.pop_size
        counts = np.zeros(p.pop_size, dtype=np.int64)
        start = 0
        if p.elitism:
            e = argbest(E)
            new[0], newE[0] = pop[e].copy(), E[e]
            start = 1
        for j in range(start, p.pop_size):
            a = tournament(E, p, run, gen, j, 0)
            b = tournament(E, p, run, gen, j, 1)
            child = crossover(pop[a], pop[b], lig, p, run, gen, j)
            child = mutate(child, lig, p, run, gen, j)
            new[j], newE[j] = child, energy(grid, lig, child)
            counts[j] += 1
        if n_ls:
            for i in local_search_picks(p, run, gen):
                if p.ls_method == "solis_wets":
                    bx, be = local_search_sw(grid, lig, new[i], p.ls_iters, p.seed, run, gen, i)
                else:
                    bx, be = local_search(grid, lig, new[i], p.ls_iters, p.rho, p.eps)
                new[i], newE[i] = bx, be
                counts[i] += p.ls_iters
        evals += int(counts.sum())
        pop, E = new, newE
        if trace is not None:
            trace.append(dict(gen=gen, genes=np.array(pop), energy=np.array(E), evals=evals))
    b = argbest(E)
    return pop[b].copy(), E[b], evals, gen


def lga_dock(grid, lig, p: DockParams):
    """All runs; results sorted by energy (ties to the lower run index)."""
    res = [run_lga(grid, lig, p, r) for r in range(p.n_runs)]
    order = sorted(range(p.n_runs), key=lambda r: (res[r][1], r))
    return dict(order=order,
                best_energy=np.array([res[r][1] for r in order]),
                best_genes=np.array([res[r][0] for r in order]),
                evals=np.array([res[r][2] for r in order]),
                generations=np.array([res[r][3] for r in order]))
