"""Solis-Wets local search on the genotype (oracle; test infrastructure only).

The paper names Solis and Wets' random search ("Minimization by random search techniques",
Mathematics of Operations Research 6(1), 1981) as the miniapp's local optimiser (Background,
"Design and Structure of MiniMDock").  This is their adaptive random search with a bias term:
from the current point x with energy E, draw a step xi ~ N(b, (rho sigma)^2) per gene; if
E(x + xi) < E move there and set b <- 0.2 b + 0.4 xi; otherwise, if E(x - xi) < E move there and
set b <- b - 0.4 xi; otherwise set b <- 0.5 b.  After `expand_after` successes in a row rho is
multiplied by `expand`, after `contract_after` failures in a row by `contract`.

Readings taken here (the paper gives no parameter):
  * per-gene deviation scales sigma: 0.5 A for translation, 0.05 for each quaternion component,
    0.25 rad for each torsion; rho starts at 1 and is kept within [0.01, 4]; expansion x2 after
    4 successes, contraction x0.5 after 4 failures (the AutoDock lineage's usual counts);
  * the search spends exactly `n_evals` energy evaluations: one at the start point, then one or
    two per step (the step that would need an evaluation past the budget is not taken), so the
    evaluation count -- and with it the GA's generation count -- is known in advance;
  * after a move the quaternion is renormalised and the torsions wrapped to (-pi, pi], as in the
    gradient search; the result is the final point (it only moves to strictly lower energies);
  * normals: Box-Muller, z = sqrt(-2 ln u1) cos(2 pi u2) with u1 = (k1 + 1) / 2^24 and
    u2 = k2 / 2^24 for 24-bit counter-based draws k1 (index 2m) and k2 (index 2m + 1), m being
    64 x step + gene.
"""
from __future__ import annotations

import math

import numpy as np

from . import rng as R
from .adadelta import project_genes
from .scoring import energy

SIGMA_TRANS = 0.5
SIGMA_QUAT = 0.05
SIGMA_TORS = 0.25
RHO0, RHO_MIN, RHO_MAX = 1.0, 0.01, 4.0
EXPAND, CONTRACT = 2.0, 0.5
EXPAND_AFTER, CONTRACT_AFTER = 4, 4


def sigmas(n_genes):
    s = np.full(n_genes, SIGMA_TORS)
    s[0:3] = SIGMA_TRANS
    s[3:7] = SIGMA_QUAT
    return s


def box_muller(k1: int, k2: int) -> float:
    """A standard normal from two 24-bit integers."""
    u1 = (k1 + 1) / 16777216.0
    u2 = k2 / 16777216.0
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def counter_normals(seed, run, gen, indiv):
    """normals(step, gene) for one local search, from the counter-based generator."""
    def normal(step, gene):
        m = 64 * step + gene
        return box_muller(R.draw_u24(seed, run, gen, indiv, R.P_LS_SW, 2 * m),
                          R.draw_u24(seed, run, gen, indiv, R.P_LS_SW, 2 * m + 1))
    return normal


def solis_wets(f, x0, n_evals, normal, sigma, project=lambda x: x, record=None):
    """Generic Solis-Wets minimisation of f from x0 with exactly n_evals evaluations of f.
    normal(step, i) gives the i-th standard normal of a step; project(x) maps a moved point back
    onto the parameter domain.  record (a list) receives one dict per step: the step, the
    deviation xi, which side succeeded (+1, -1, 0), rho and b after the step.
    Returns (x, f(x), trace of every evaluated energy)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    n = x.size
    e = f(x)
    trace = [e]
    b = np.zeros(n)
    rho = RHO0
    succ = fail = 0
    step = 0
    while len(trace) < n_evals:
        xi = np.array([b[i] + rho * sigma[i] * normal(step, i) for i in range(n)])
        x1 = project(x + xi)
        e1 = f(x1)
        trace.append(e1)
        side = 0
        if e1 < e:
            x, e, side = x1, e1, 1
            b = 0.2 * b + 0.4 * xi
        elif len(trace) < n_evals:
            x2 = project(x - xi)
            e2 = f(x2)
            trace.append(e2)
            if e2 < e:
                x, e, side = x2, e2, -1
                b = b - 0.4 * xi
            else:
                b = 0.5 * b
        else:
            b = 0.5 * b
        if side:
            succ, fail = succ + 1, 0
        else:
            succ, fail = 0, fail + 1
        if succ >= EXPAND_AFTER:
            rho, succ = min(RHO_MAX, rho * EXPAND), 0
        if fail >= CONTRACT_AFTER:
            rho, fail = max(RHO_MIN, rho * CONTRACT), 0
        if record is not None:
            record.append(dict(step=step, xi=xi, side=side, rho=rho, b=b.copy()))
        step += 1
    return x, e, trace


def local_search_sw(grid, lig, genes0, n_evals, seed, run=0, gen=0, indiv=0, trace=False, points=None):
    """Solis-Wets on a ligand's genotype; returns (genes, energy[, energies of every evaluation]).
    points (a list) receives every evaluated genotype, in order."""
    def f(g):
        if points is not None:
            points.append(g.copy())
        return energy(grid, lig, g)
    x, e, tr = solis_wets(f, genes0, n_evals,
                          counter_normals(seed, run, gen, indiv), sigmas(lig.n_genes),
                          project=lambda g: project_genes(g, lig.n_torsions))
    if trace:
        return x, e, tr
    return x, e
