"""Pins for the Solis-Wets oracle: a hand-worked trajectory with scripted normals, the step-size
rules, the evaluation budget, Box-Muller's closed form and moments, convergence on closed-form
minima, and the docking wrapper's projection and bookkeeping."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import lga as OG
from oracle import ligand as OL
from oracle import scoring as S
from oracle import solis_wets as SW
from workload import synth


def _scripted(zs):
    """normal(step, i) returning zs[step] (one-dimensional searches)."""
    return lambda step, i: zs[step]


HAND_ZS = [-1.0, 0.5, 3.0, -0.1, 0.0, 0.0]


def test_hand_worked_trajectory():
    """f(x) = x^2 from x0 = 2, sigma 1, scripted normals -1, 0.5, 3, -0.1 (worked by hand):
      step 0: xi = -1            -> x = 1 accepted (f 1),              b = -0.4
      step 1: xi = -0.4 + 0.5 = 0.1 -> 1.1 rejected (1.21), 0.9 accepted (0.81), b = -0.44
      step 2: xi = -0.44 + 3 = 2.56 -> 3.46 (11.9716), -1.66 (2.7556) both rejected, b = -0.22
      step 3: xi = -0.22 - 0.1 = -0.32 -> 0.58 accepted (0.3364),    b = -0.172"""
    f = lambda x: float(x[0] ** 2)
    rec = []
    x, e, tr = SW.solis_wets(f, [2.0], 7, _scripted(HAND_ZS), [1.0], record=rec)
    assert np.allclose(tr, [4, 1, 1.21, 0.81, 11.9716, 2.7556, 0.3364], rtol=0, atol=1e-12)
    assert abs(x[0] - 0.58) < 1e-12 and abs(e - 0.3364) < 1e-12
    assert [r["side"] for r in rec] == [1, -1, 0, 1]
    assert np.allclose([r["b"][0] for r in rec], [-0.4, -0.44, -0.22, -0.172], atol=1e-12)
    assert np.allclose([r["xi"][0] for r in rec], [-1, 0.1, 2.56, -0.32], atol=1e-12)
    assert all(r["rho"] == 1.0 for r in rec)


@pytest.mark.parametrize("n_evals,x_end,e_end", [(1, 2.0, 4.0), (2, 1.0, 1.0), (3, 1.0, 1.0),
                                                 (4, 0.9, 0.81), (5, 0.9, 0.81), (6, 0.9, 0.81)])
def test_budget_is_exact(n_evals, x_end, e_end):
    """Exactly n_evals evaluations; a step cut short by the budget tries only x + xi."""
    calls = []

    def f(x):
        calls.append(float(x[0]))
        return float(x[0] ** 2)
    x, e, tr = SW.solis_wets(f, [2.0], n_evals, _scripted(HAND_ZS), [1.0])
    assert len(calls) == len(tr) == n_evals
    assert abs(x[0] - x_end) < 1e-12 and abs(e - e_end) < 1e-12


def test_contraction_and_floor():
    """A flat function never improves: rho halves after every 4 failures, down to 0.01, and the
    bias stays zero."""
    rec = []
    steps = 40
    SW.solis_wets(lambda x: 0.0, np.zeros(3), 1 + 2 * steps, lambda s, i: 0.7, np.ones(3), record=rec)
    rhos = [r["rho"] for r in rec]
    expect, rho = [], 1.0
    for k in range(1, steps + 1):
        if k % 4 == 0:
            rho = max(0.01, rho / 2)
        expect.append(rho)
    assert rhos == expect
    assert rhos[-1] == 0.01 and 0.0078125 not in rhos
    assert all(not r["b"].any() and r["side"] == 0 for r in rec)


def test_expansion_and_cap():
    """f(x) = -x with positive normals always succeeds on the + side: rho doubles after every 4
    successes up to 4, and the bias follows b <- 0.2 b + 0.4 xi."""
    rec = []
    SW.solis_wets(lambda x: -float(x[0]), [0.0], 21, lambda s, i: 1.0, [1.0], record=rec)
    assert [r["side"] for r in rec] == [1] * 20
    assert [r["rho"] for r in rec] == [1.0] * 3 + [2.0] * 4 + [4.0] * 13
    b, rho = 0.0, 1.0
    for k, r in enumerate(rec):
        xi = b + rho * 1.0
        b = 0.2 * b + 0.4 * xi
        assert abs(r["xi"][0] - xi) < 1e-12 and abs(r["b"][0] - b) < 1e-12
        if k in (3, 7, 11, 15, 19):
            rho = min(4.0, 2 * rho)


def test_box_muller_closed_form():
    assert SW.box_muller(2 ** 24 - 1, 0) == 0.0                      # u1 = 1
    assert abs(SW.box_muller(0, 0) - math.sqrt(48 * math.log(2))) < 1e-12   # u1 = 2^-24
    assert abs(SW.box_muller(0, 2 ** 23) + math.sqrt(48 * math.log(2))) < 1e-12  # cos(pi) = -1
    assert abs(SW.box_muller(2 ** 22, 2 ** 22)) < 1e-9               # cos(pi/2) = 0


def test_counter_normals_are_standard():
    nrm = SW.counter_normals(seed=9, run=1, gen=2, indiv=3)
    z = np.array([nrm(s, i) for s in range(160) for i in range(64)])
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # different individuals and generations draw different numbers
    other = SW.counter_normals(seed=9, run=1, gen=2, indiv=4)
    assert nrm(0, 0) != other(0, 0)


def test_converges_on_a_quadratic():
    rng = np.random.default_rng(3)
    c = rng.normal(size=5)
    f = lambda x: float(np.sum((x - c) ** 2))
    nrm = lambda s, i: float(np.random.default_rng([s, i]).standard_normal())
    x, e, tr = SW.solis_wets(f, c + 3.0, 3000, nrm, np.full(5, 0.5))
    assert e < 1e-3 and np.linalg.norm(x - c) < 0.05
    acc = [tr[0]]
    for t in tr[1:]:
        if t < acc[-1]:
            acc.append(t)
    assert e == min(tr) == acc[-1]


def _grid(n=24, seed=13):
    rec = synth.make_receptor(n, seed)
    return S.make_grid(rec.maps, rec.origin, rec.spacing)


def test_docking_wrapper_projects_and_reports(type_params):
    g = _grid()
    lig = OL.from_synth(synth.make_ligand(10, 3, 5, type_params))
    r = np.random.default_rng(5)
    x0 = np.concatenate([r.uniform(-1, 1, 3), r.normal(size=4), r.uniform(-3, 3, 3)])
    x0[3:7] /= np.linalg.norm(x0[3:7])
    x, e, tr = SW.local_search_sw(g, lig, x0, 200, seed=4, indiv=2, trace=True)
    assert len(tr) == 200 and tr[0] == S.energy(g, lig, x0)
    assert e == min(tr) and e < tr[0]
    assert abs(S.energy(g, lig, x) - e) < 1e-12
    assert abs(np.linalg.norm(x[3:7]) - 1) < 1e-12
    assert np.all(x[7:] > -math.pi) and np.all(x[7:] <= math.pi)
    x2, e2 = SW.local_search_sw(g, lig, x0, 200, seed=4, indiv=2)
    assert e2 == e and np.array_equal(x2, x)
    _, e3 = SW.local_search_sw(g, lig, x0, 200, seed=4, indiv=3)
    assert e3 != e


def test_one_atom_finds_the_well(type_params):
    """One atom in a quadratic bowl sampled on the grid: the search reaches the bottom."""
    n, h = 24, 0.375
    origin = np.full(3, -0.5 * (n - 1) * h)
    ax = origin[0] + h * np.arange(n)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    bowl = 0.5 * ((x - 0.6) ** 2 + (y + 0.3) ** 2 + (z - 0.1) ** 2)
    maps = np.zeros((9, n, n, n))
    maps[:] = bowl
    g = S.make_grid(maps, origin, h)
    lig = OL.prepare(np.zeros((1, 3)), [0], [0.0], np.zeros((0, 2), int), np.zeros(0, int), type_params)
    bx, be = SW.local_search_sw(g, lig, np.array([-2.0, 2.0, 1.5, 1, 0, 0, 0]), 600, seed=1)
    assert np.linalg.norm(bx[0:3] - np.array([0.6, -0.3, 0.1])) < 0.3
    assert be < 0.1


def test_lga_with_solis_wets(type_params):
    """The GA with Solis-Wets keeps its invariants and spends ls_iters per searched individual."""
    g = _grid()
    lig = OL.from_synth(synth.make_ligand(8, 2, 9, type_params))
    p = OG.DockParams(n_runs=1, pop_size=20, max_generations=4, ls_rate=0.2, ls_iters=25, seed=3,
                      ls_method="solis_wets")
    trace = []
    bx, be, evals, gens = OG.run_lga(g, lig, p, 0, trace=trace)
    best = [t["energy"].min() for t in trace]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    assert evals == p.pop_size + gens * OG.evals_per_generation(p) == 20 + 4 * (19 + 4 * 25)
    for t in trace:
        for x, e in zip(t["genes"], t["energy"]):
            assert abs(S.energy(g, lig, x) - e) < 1e-9
    pa = OG.DockParams(**{**p.__dict__, "ls_method": "adadelta"})
    _, be_a, _, _ = OG.run_lga(g, lig, pa, 0)
    assert be_a != be
