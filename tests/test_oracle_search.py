"""Pins of the oracle's ADADELTA local search and Lamarckian GA."""
import math

import numpy as np
import pytest
import torch

from oracle import adadelta as OA
from oracle import lga as OG
from oracle import ligand as OL
from oracle import scoring as S
from workload import synth


def test_adadelta_first_step_closed_form():
    rho, eps = 0.8, 1e-2
    g = np.array([3.0, -0.5, 1e-3, 0.0, 40.0])
    x1, eg2, edx2 = OA.adadelta_step(np.zeros(5), g, np.zeros(5), np.zeros(5), rho, eps)
    want = -math.sqrt(eps) / np.sqrt((1 - rho) * g * g + eps) * g
    assert np.allclose(x1, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("rho,eps", [(0.8, 1e-2), (0.95, 1e-6)])
def test_adadelta_matches_torch_on_rosenbrock(rho, eps):
    """Our update against torch.optim.Adadelta(lr=1) in float64 on an analytic function."""
    def grad(p):
        x, y = p
        return np.array([-2 * (1 - x) - 400 * x * (y - x * x), 200 * (y - x * x)])

    p = np.array([-1.2, 1.0])
    eg2 = np.zeros(2)
    edx2 = np.zeros(2)
    tp = torch.tensor([-1.2, 1.0], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adadelta([tp], lr=1.0, rho=rho, eps=eps)
    for _ in range(300):
        g = grad(p)
        p, eg2, edx2 = OA.adadelta_step(p, g, eg2, edx2, rho, eps)
        opt.zero_grad()
        tx, ty = tp[0], tp[1]
        ((1 - tx) ** 2 + 100 * (ty - tx * tx) ** 2).backward()
        opt.step()
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def _grid(n=24, seed=13):
    rec = synth.make_receptor(n, seed)
    return S.make_grid(rec.maps, rec.origin, rec.spacing)


def test_local_search_keeps_best_and_projects(type_params):
    g = _grid()
    lig = OL.from_synth(synth.make_ligand(10, 3, 5, type_params))
    r = np.random.default_rng(5)
    x0 = np.concatenate([r.uniform(-1, 1, 3), r.normal(size=4), r.uniform(-3, 3, 3)])
    x0[3:7] /= np.linalg.norm(x0[3:7])
    bx, be, traj = OA.local_search(g, lig, x0, iters=60, trace=True)
    es = np.array([e for e, _ in traj])
    assert be == es.min()
    assert np.array_equal(bx, traj[int(np.argmin(es))][1])       # first of equal minima
    assert be <= S.energy(g, lig, x0)
    assert abs(S.energy(g, lig, bx) - be) < 1e-12
    for _, x in traj:
        assert abs(np.linalg.norm(x[3:7]) - 1.0) < 1e-12
        assert np.all(x[7:] > -math.pi) and np.all(x[7:] <= math.pi)
    assert traj[0][0] == S.energy(g, lig, x0)


def test_local_search_descends_a_smooth_well(type_params):
    """One atom in a quadratic bowl sampled on the grid: ADADELTA walks to the bottom cell."""
    n, h = 24, 0.375
    origin = np.full(3, -0.5 * (n - 1) * h)
    ax = origin[0] + h * np.arange(n)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    bowl = 0.5 * ((x - 0.6) ** 2 + (y + 0.3) ** 2 + (z - 0.1) ** 2)
    maps = np.zeros((9, n, n, n))
    maps[:] = bowl
    g = S.make_grid(maps, origin, h)
    lig = OL.prepare(np.zeros((1, 3)), [0], [0.0], np.zeros((0, 2), int), np.zeros(0, int), type_params)
    bx, be = OA.local_search(g, lig, np.array([-2.0, 2.0, 1.5, 1, 0, 0, 0]), iters=300)
    assert np.linalg.norm(bx[0:3] - np.array([0.6, -0.3, 0.1])) < 0.3
    assert be < 0.1


# ------------------------------------------------------------------ LGA
def test_eval_budget_closed_form():
    p = OG.DockParams(n_runs=1, pop_size=150, max_generations=10, ls_rate=0.06, ls_iters=300)
    assert OG.n_local_search(p) == 9
    assert OG.planned_generations(p) == 10
    assert 150 + 10 * OG.evals_per_generation(p) == 28640
    p2 = OG.DockParams(pop_size=150, max_generations=10 ** 6, max_evals_per_run=2_500_000,
                       ls_rate=1.0, ls_iters=300)
    assert OG.evals_per_generation(p2) == 45149
    assert OG.planned_generations(p2) == 56


def test_ls_picks_distinct_and_counted():
    p = OG.DockParams(pop_size=150, ls_rate=0.06)
    for gen in range(1, 6):
        picks = OG.local_search_picks(p, 0, gen)
        assert len(picks) == 9 and len(set(picks)) == 9
    assert OG.local_search_picks(p, 0, 1) != OG.local_search_picks(p, 0, 2)


def _small_dock(type_params, lig, g, **kw):
    p = OG.DockParams(n_runs=1, pop_size=20, max_generations=4, ls_rate=0.2, ls_iters=15, seed=3)
    for k, v in kw.items():
        setattr(p, k, v)
    trace = []
    bx, be, evals, gens = OG.run_lga(g, lig, p, 0, trace=trace)
    return p, trace, bx, be, evals, gens


def test_lga_invariants(type_params):
    g = _grid()
    lig = OL.from_synth(synth.make_ligand(8, 2, 9, type_params))
    p, trace, bx, be, evals, gens = _small_dock(type_params, lig, g)
    best = [t["energy"].min() for t in trace]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))           # elitism + Lamarckian LS
    for prev, cur in zip(trace, trace[1:]):
        e = OG.argbest(prev["energy"])
        assert np.array_equal(cur["genes"][0], prev["genes"][e]) or cur["energy"][0] <= prev["energy"][e]
    assert evals == p.pop_size + gens * OG.evals_per_generation(p)
    for t in trace:
        for x, e in zip(t["genes"], t["energy"]):
            assert abs(S.energy(g, lig, x) - e) < 1e-9
            assert abs(np.linalg.norm(x[3:7]) - 1.0) < 1e-9
    assert be == best[-1]
    # deterministic given the seed
    _, trace2, bx2, be2, _, _ = _small_dock(type_params, lig, g)
    assert be2 == be and np.array_equal(bx2, bx)


def _well_grid(n=16, h=0.375, seed=4):
    """A small receptor whose nine maps are 2 minus four Gaussian wells each (depths 1-4,
    width 1 A, centres inside the box): smooth fields with distinct minima.  (The synthetic
    receptor recipe clips to a constant +10 everywhere in a box this small.)"""
    rng = np.random.default_rng(seed)
    ax = np.arange(n) * h
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    maps = np.zeros((9, n, n, n))
    for m in range(9):
        f = np.full((n, n, n), 2.0)
        for _ in range(4):
            c = rng.uniform(0.8, (n - 1) * h - 0.8, 3)
            a = rng.uniform(1.0, 4.0)
            f -= a * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 2.0)
        maps[m] = f
    return S.make_grid(maps, np.zeros(3), h)


def _fibonacci_rotations(n):
    """Rotations taking +x to n near-uniform directions (Fibonacci sphere)."""
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    r = np.sqrt(1 - z * z)
    ph = math.pi * (1 + 5 ** 0.5) * i
    out = []
    for d in np.stack([r * np.cos(ph), r * np.sin(ph), z], 1):
        v = np.cross([1.0, 0.0, 0.0], d)
        sn, cs = np.linalg.norm(v), d[0]
        K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]]) / max(sn, 1e-300)
        th = math.atan2(sn, cs)
        out.append(np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K)
    return out


def _lattice_minimum(g, lig, rotations, step):
    """Brute force: the lowest energy of the rigid ligand over every orientation given and every
    translation on a lattice of `step` A over the box."""
    from oracle import pose as OP
    p0 = OP.pose(lig, np.r_[0, 0, 0, 1, 0, 0, 0])
    lo, hi = g.origin, g.origin + (g.n_xyz - 1) * g.spacing
    T = np.stack(np.meshgrid(*[np.arange(lo[a], hi[a] + 1e-9, step) for a in range(3)], indexing="ij"),
                 -1).reshape(-1, 3)
    best = np.inf
    for Rm in rotations:
        X = (T[:, None, :] + (p0 @ Rm.T)[None, :, :]).reshape(-1, 3)
        e, _, _ = S.grid_energies(g, X, np.tile(lig.types, T.shape[0]), np.tile(lig.charges, T.shape[0]))
        best = min(best, float(e.reshape(T.shape[0], -1).sum(1).min()))
    return best


SMALL_LIGANDS = [(1, [2], [-0.2], [[0, 0, 0]]),
                 (2, [2, 5], [-0.2, 0.2], [[-0.75, 0, 0], [0.75, 0, 0]]),
                 (3, [1, 3, 6], [-0.3, 0.1, 0.2], [[-1.2, -0.3, 0], [0, 0.6, 0], [1.2, -0.3, 0]])]


@pytest.mark.parametrize("case", SMALL_LIGANDS, ids=["1atom", "2atoms", "3atoms"])
def test_lga_small_ligands_reach_lattice_minimum(type_params, case):
    """On 1-3-atom (rigid, pair-free) ligands the energy is a sum of trilinear fields, so two
    bounds hold exactly: the LGA's best is never below the sum of the per-atom field minima,
    and a brute-force lattice over orientations and translations gives a reference the search
    must reach within 1 % of the fields' spread.  For one atom the lattice (every node) is the
    exact minimum, since a trilinear interpolant is extreme at a node."""
    from scipy.spatial.transform import Rotation
    na, types, q, xyz = case
    g = _well_grid()
    bonds = np.array([[k, k + 1] for k in range(na - 1)], int).reshape(-1, 2)
    lig = OL.prepare(np.array(xyz, float), types, q, bonds, np.zeros(0, int), type_params)
    fields = [g.maps[t] + c * g.maps[7] + abs(c) * g.maps[8] for t, c in zip(types, q)]
    lower = sum(float(f.min()) for f in fields)
    spread = sum(float(f.max() - f.min()) for f in fields)
    if na == 1:
        ref = lower
    elif na == 2:
        ref = _lattice_minimum(g, lig, _fibonacci_rotations(100), 0.25)
    else:
        ref = _lattice_minimum(g, lig, Rotation.random(150, random_state=3).as_matrix(), 0.25)
    p = OG.DockParams(n_runs=2, pop_size=30, max_generations=8, ls_rate=0.3, ls_iters=40, seed=5)
    res = OG.lga_dock(g, lig, p)
    best = float(res["best_energy"][0])
    assert best >= lower - 1e-9
    assert best <= ref + 0.01 * spread, (best, ref, spread)
    assert res["best_energy"][0] <= res["best_energy"][1]


def test_initial_individual_distribution(type_params):
    """The initial population's sampler draws what it states: translation uniform over the box
    [o, o + (n - 1) h] per axis, orientation uniform over rotations (Haar measure: rotation angle
    density (1 - cos a) / pi, axis uniform on the sphere) and torsions uniform in (-pi, pi] --
    Kolmogorov-Smirnov tests on 6000 draws; the same tests reject a sampler that normalises a
    uniform 4-cube point, which is not uniform over rotations."""
    from scipy import stats
    g = _well_grid()
    lig = OL.from_synth(synth.make_ligand(8, 3, 5, type_params))
    p = OG.DockParams(seed=123)
    X = np.array([OG.initial_individual(g, lig, p, run, i) for run in range(3) for i in range(2000)])
    lo, hi = g.origin, g.origin + (g.n_xyz - 1) * g.spacing
    assert np.all(X[:, 0:3] >= lo) and np.all(X[:, 0:3] <= hi)
    for a in range(3):
        assert stats.kstest((X[:, a] - lo[a]) / (hi[a] - lo[a]), "uniform").pvalue > 1e-3
    assert np.allclose(np.linalg.norm(X[:, 3:7], axis=1), 1.0, atol=1e-12)

    def haar_pvalues(Q):
        w = np.clip(np.abs(Q[:, 0]), 0.0, 1.0)
        ang = 2.0 * np.arccos(w)                          # rotation angle in [0, pi]
        p_ang = stats.kstest(ang, lambda a: (a - np.sin(a)) / math.pi).pvalue
        v = Q[:, 1:4] * np.sign(Q[:, :1] + 1e-300)
        axis = v / np.linalg.norm(v, axis=1, keepdims=True)
        p_axis = stats.kstest((axis[:, 2] + 1) / 2, "uniform").pvalue   # Archimedes: z uniform
        return p_ang, p_axis

    p_ang, p_axis = haar_pvalues(X[:, 3:7])
    assert p_ang > 1e-3 and p_axis > 1e-3
    for k in range(lig.n_torsions):
        t = X[:, 7 + k]
        assert np.all(t > -math.pi) and np.all(t <= math.pi)
        assert stats.kstest((t + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    # power: a plausible wrong sampler is rejected
    cube = np.random.default_rng(0).uniform(-1, 1, (6000, 4))
    cube /= np.linalg.norm(cube, axis=1, keepdims=True)
    assert min(haar_pvalues(cube)) < 1e-3


def test_mutation_and_crossover_units(type_params):
    lig = OL.from_synth(synth.make_ligand(12, 4, 3, type_params))
    p = OG.DockParams(seed=11, mutation_rate=1.0, crossover_rate=1.0)
    xa = np.concatenate([[1.0, 2.0, 3.0], [1, 0, 0, 0], [0.1, 0.2, 0.3, 0.4]])
    xb = np.concatenate([[-1.0, -2.0, -3.0], [0, 1, 0, 0], [-0.1, -0.2, -0.3, -0.4]])
    for slot in range(30):
        c = OG.crossover(xa, xb, lig, p, 0, 1, slot)
        # each unit comes whole from one parent
        assert c[3:7].tolist() in (xa[3:7].tolist(), xb[3:7].tolist())
        for k in list(range(3)) + list(range(7, 11)):
            assert c[k] in (xa[k], xb[k])
        m = OG.mutate(xa, lig, p, 0, 1, slot)
        assert np.all(np.abs(m[0:3] - xa[0:3]) <= 2.0)
        assert abs(np.linalg.norm(m[3:7]) - 1.0) < 1e-12
        # the quaternion moved by at most pi/2 of rotation angle
        ang = 2 * math.acos(min(1.0, abs(m[3])))
        assert ang <= math.pi / 2 + 1e-9
        assert np.all(m[7:] > -math.pi) and np.all(m[7:] <= math.pi)


def test_tournament_better_wins_at_stated_rate():
    """Binary tournament: of two distinct picks the lower-energy one wins with probability
    tournament_rate (0.6)."""
    p = OG.DockParams(pop_size=150, seed=21)
    E = np.random.default_rng(0).normal(size=150)
    wins = total = 0
    for slot in range(4000):
        a = OG.R.randint(150, p.seed, 0, 1, slot, OG.R.P_TOURNAMENT, 0)
        b = OG.R.randint(150, p.seed, 0, 1, slot, OG.R.P_TOURNAMENT, 1)
        if a == b:
            continue
        w = OG.tournament(E, p, 0, 1, slot, 0)
        total += 1
        wins += int(w == (a if E[a] < E[b] else b))
    assert abs(wins / total - 0.6) < 0.03


def test_mutation_and_crossover_rates(type_params):
    lig = OL.from_synth(synth.make_ligand(12, 4, 3, type_params))
    p = OG.DockParams(seed=5)
    xa = np.concatenate([[1.0, 2.0, 3.0], [1, 0, 0, 0], [0.1, 0.2, 0.3, 0.4]])
    xb = np.concatenate([[-1.0, -2.0, -3.0], [0, 1, 0, 0], [-0.1, -0.2, -0.3, -0.4]])
    changed = units = same_as_a = 0
    n = 3000
    for slot in range(n):
        m = OG.mutate(xa, lig, p, 0, 2, slot)
        changed += int(np.sum(m[0:3] != xa[0:3])) + int(np.any(m[3:7] != xa[3:7])) + int(np.sum(m[7:] != xa[7:]))
        units += 8
        c = OG.crossover(xa, xb, lig, p, 0, 2, slot)
        same_as_a += int(np.array_equal(c, xa))
    assert abs(changed / units - 0.02) < 0.006
    # child == parent A unless crossover happens with lo < hi: P = 0.2 + 0.8 * P(c1 == c2) = 0.2 + 0.8/9
    assert abs(same_as_a / n - (0.2 + 0.8 / 9)) < 0.03
