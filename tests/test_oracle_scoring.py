"""Pins of the oracle's energy and genotype gradient."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator
from scipy.spatial.transform import Rotation

from oracle import constants as C
from oracle import ligand as OL
from oracle import pose as OP
from oracle import scoring as S
from workload import synth


def _grid(n=12, seed=3, h=0.375):
    rec = synth.make_receptor(n, seed, spacing=h)
    return S.make_grid(rec.maps, rec.origin, rec.spacing)


# ------------------------------------------------------------------ trilinear
def test_trilinear_exact_at_nodes():
    g = _grid()
    vol = g.maps[2]
    r = np.random.default_rng(0)
    for _ in range(50):
        i = r.integers(0, 11, 3)
        v, _ = S.trilinear(vol, i.astype(float))
        assert v == vol[i[2], i[1], i[0]]


def test_trilinear_exact_for_linear_field():
    n = 9
    a, b, c, d = 0.7, -1.3, 2.1, 0.4
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    vol = a * x + b * y + c * z + d
    r = np.random.default_rng(1)
    for _ in range(100):
        p = r.uniform(0, n - 1 - 1e-9, 3)
        v, dv = S.trilinear(vol, p)
        assert abs(v - (a * p[0] + b * p[1] + c * p[2] + d)) < 1e-12
        assert np.allclose(dv, [a, b, c], atol=1e-12)


def test_trilinear_constant_field_zero_gradient():
    vol = np.full((5, 6, 7), 3.25)
    v, dv = S.trilinear(vol, np.array([2.3, 1.7, 0.2]))
    assert abs(v - 3.25) < 1e-14 and np.all(np.abs(dv) < 1e-14)


def test_trilinear_matches_scipy():
    g = _grid(10, 5)
    vol = g.maps[7]
    nz, ny, nx = vol.shape
    interp = RegularGridInterpolator((np.arange(nz), np.arange(ny), np.arange(nx)), vol, method="linear")
    r = np.random.default_rng(2)
    for _ in range(200):
        p = r.uniform(0, 9 - 1e-9, 3)
        v, _ = S.trilinear(vol, p)
        assert abs(v - interp([[p[2], p[1], p[0]]])[0]) < 1e-12


def test_trilinear_gradient_fd_inside_cell():
    g = _grid(10, 6)
    vol = g.maps[0]
    r = np.random.default_rng(3)
    for _ in range(50):
        cell = r.integers(0, 8, 3)
        p = cell + r.uniform(0.05, 0.95, 3)
        _, dv = S.trilinear(vol, p)
        h = 1e-6
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (S.trilinear(vol, p + e)[0] - S.trilinear(vol, p - e)[0]) / (2 * h)
            assert abs(fd - dv[a]) < 1e-6 * max(1.0, abs(dv[a]))


def test_atom_grid_energy_roles_and_outside():
    g = _grid(10, 7)
    x = g.origin + g.spacing * np.array([3.25, 4.5, 2.75])
    e, dedx, _ = S.atom_grid_energy(g, x, 2, -0.3)
    gp = (x - g.origin) / g.spacing
    want = S.trilinear(g.maps[2], gp)[0] - 0.3 * S.trilinear(g.maps[7], gp)[0] + 0.3 * S.trilinear(g.maps[8], gp)[0]
    assert abs(e - want) < 1e-12
    # outside: constant penalty plus K d^2 to the box, restoring gradient
    hi = g.origin + (g.n_xyz - 1) * g.spacing
    xo = hi + np.array([0.5, -1.0, 0.0]) * np.array([1, 0, 0]) + np.array([0, -1.0, 0])
    e, dedx, _ = S.atom_grid_energy(g, xo, 1, 0.2)
    d = xo - np.clip(xo, g.origin, hi)
    assert abs(e - (C.P_OUT + C.K_OUT * d @ d)) < 1e-9
    assert np.allclose(dedx, 2 * C.K_OUT * d)
    # the last grid plane counts as outside
    xl = g.origin + g.spacing * np.array([9.0, 3.0, 3.0])
    assert not S.inside(g, xl)[0]


# ------------------------------------------------------------------ pair terms
def test_lj_12_6_minimum():
    eps, R = 0.17, 3.6
    c12, c6 = eps * R ** 12, 2 * eps * R ** 6
    e, dedr, _, _ = S.pair_energy(R, False, c12, c6, 0.0, 0.0)
    assert abs(e - (-C.W_VDW * eps)) < 1e-12
    assert abs(dedr) < 1e-12
    assert S.pair_energy(R * 0.99, False, c12, c6, 0, 0)[0] > e
    assert S.pair_energy(R * 1.01, False, c12, c6, 0, 0)[0] > e


def test_hb_12_10_minimum():
    eps, R = 4.0, 1.9
    c12, c10 = 5 * eps * R ** 12, 6 * eps * R ** 10
    e, dedr, _, _ = S.pair_energy(R, True, c12, c10, 0.0, 0.0)
    assert abs(e - (-C.W_HB * eps)) < 1e-12
    assert abs(dedr) < 1e-10


def test_dielectric_limits():
    eps0, _ = S.dielectric(0.0)
    assert abs(eps0 - (C.DIEL_A + C.DIEL_B / (1 + C.DIEL_K))) < 1e-12
    epsinf, _ = S.dielectric(1e4)
    assert abs(epsinf - 78.4) < 1e-9
    for r in (0.7, 3.0, 10.0):
        h = 1e-6
        fd = (S.dielectric(r + h)[0] - S.dielectric(r - h)[0]) / (2 * h)
        assert abs(fd - S.dielectric(r)[1]) < 1e-7


def test_coulomb_and_desolvation_closed_forms():
    r = 4.0
    eps, _ = S.dielectric(r)
    e, _, _, (elj, eel, eds) = S.pair_energy(r, False, 0.0, 0.0, -0.12, 0.0)
    assert abs(eel - C.W_EL * C.COULOMB * -0.12 / (r * eps)) < 1e-13
    e, _, _, (elj, eel, eds) = S.pair_energy(r, False, 0.0, 0.0, 0.0, 2.5)
    assert abs(eds - C.W_DS * 2.5 * math.exp(-r * r / (2 * C.DESOLV_SIGMA ** 2))) < 1e-13
    # r -> 0 is clamped to R_MIN, with zero gradient
    e0, d0, _, (_, _, eds0) = S.pair_energy(0.0, False, 1.0, 1.0, 0.1, 2.5)
    em, _, _, _ = S.pair_energy(C.R_MIN, False, 1.0, 1.0, 0.1, 2.5)
    assert e0 == em and d0 == 0.0
    assert abs(eds0 - C.W_DS * 2.5 * math.exp(-C.R_MIN ** 2 / (2 * C.DESOLV_SIGMA ** 2))) < 1e-13
    # cutoffs
    assert S.pair_energy(8.5, False, 1e6, 1e3, 0.0, 3.0)[0] == 0.0
    assert S.pair_energy(8.5, False, 0, 0, 0.1, 0)[0] != 0.0
    assert S.pair_energy(21.0, False, 0, 0, 0.1, 0)[0] == 0.0


def test_pair_derivative_fd():
    r0 = np.random.default_rng(4)
    for _ in range(100):
        r = r0.uniform(0.6, 19.0)
        if abs(r - C.CUTOFF) < 1e-3:
            continue
        args = (bool(r0.integers(2)), r0.uniform(1e3, 1e7), r0.uniform(10, 1e4),
                r0.uniform(-0.25, 0.25), r0.uniform(-0.1, 0.1))
        h = 1e-6
        fd = (S.pair_energy(r + h, *args)[0] - S.pair_energy(r - h, *args)[0]) / (2 * h)
        d = S.pair_energy(r, *args)[1]
        assert abs(fd - d) < 1e-6 * max(1.0, abs(d))


def test_pair_params_mixing_rules(type_params):
    lig = OL.from_synth(synth.make_ligand(20, 4, 1, type_params))
    tp = lig.type_params
    for (i, j) in lig.pairs:
        is_hb, c12, cn, qq, ds = S.pair_params(lig, i, j)
        ti, tj = lig.types[i], lig.types[j]
        roles = {int(tp[ti, 4]), int(tp[tj, 4])}
        assert is_hb == (roles == {C.HB_DONOR, C.HB_ACCEPTOR})
        if not is_hb:
            R = 0.5 * (tp[ti, 0] + tp[tj, 0])
            e = math.sqrt(tp[ti, 1] * tp[tj, 1])
            # the 12-6 pair has its minimum -eps_ij at R_ij
            assert abs(S.pair_energy(R, False, c12, cn, 0, 0)[0] + C.W_VDW * e) < 1e-9
        else:
            # the 12-10 pair uses the acceptor's radius and well depth: minimum there
            acc = ti if int(tp[ti, 4]) == C.HB_ACCEPTOR else tj
            R, e = tp[acc, 5], tp[acc, 6]
            assert abs(S.pair_energy(R, True, c12, cn, 0, 0)[0] + C.W_HB * e) < 1e-9
        assert abs(qq - lig.charges[i] * lig.charges[j]) < 1e-15
        si = tp[ti, 3] + C.QASP * abs(lig.charges[i])
        sj = tp[tj, 3] + C.QASP * abs(lig.charges[j])
        assert abs(ds - (si * tp[tj, 2] + sj * tp[ti, 2])) < 1e-15
    assert any(S.pair_params(lig, i, j)[0] for (i, j) in lig.pairs), "no H-bond pair exercised"


# ------------------------------------------------------------------ ligand-level
def _lig(n, t, seed, tp):
    return OL.from_synth(synth.make_ligand(n, t, seed, tp))


def _intra(lig, x):
    e = 0.0
    for (i, j) in lig.pairs:
        r = np.linalg.norm(x[i] - x[j])
        e += S.pair_energy(r, *S.pair_params(lig, i, j))[0]
    return e


def _floyd(lig):
    n = lig.n_atoms
    D = np.full((n, n), 10 ** 6)
    np.fill_diagonal(D, 0)
    for a in range(n):
        for b in lig.neighbours[a]:
            D[a, b] = 1
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


@pytest.mark.parametrize("n,t,seed", [(12, 3, 21), (20, 4, 22), (40, 8, 23)])
def test_pair_list_brute_force(n, t, seed, type_params):
    """Pair list = pairs >= 3 bonds apart that some torsion separates (independent rule:
    Floyd-Warshall distances and moving-set membership)."""
    lig = _lig(n, t, seed, type_params)
    D = _floyd(lig)
    want = set()
    for i in range(n):
        for j in range(i + 1, n):
            if D[i, j] >= 3 and any(lig.moving[k, i] != lig.moving[k, j] for k in range(lig.n_torsions)):
                want.add((i, j))
    assert set(map(tuple, lig.pairs.tolist())) == want


@pytest.mark.parametrize("n,t,seed", [(20, 4, 31), (40, 8, 32)])
def test_intra_invariant_under_rigid_motion(n, t, seed, type_params):
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    for _ in range(5):
        tors = r.uniform(-math.pi, math.pi, lig.n_torsions)
        g1 = np.concatenate([r.normal(size=3) * 4, r.normal(size=4), tors])
        g2 = np.concatenate([r.normal(size=3) * 4, r.normal(size=4), tors])
        e1, e2 = _intra(lig, OP.pose(lig, g1)), _intra(lig, OP.pose(lig, g2))
        assert abs(e1 - e2) <= 1e-12 * max(1.0, abs(e1))


def test_intra_permutation_invariant(type_params):
    base = synth.make_ligand(25, 6, 41, type_params)
    lig = OL.from_synth(base)
    r = np.random.default_rng(41)
    perm = r.permutation(25)
    inv = np.argsort(perm)       # new index of old atom a is inv[a]
    xyz = base.xyz[perm]
    bonds = inv[base.bonds]
    lig2 = OL.prepare(xyz, base.types[perm], base.charges[perm], bonds, base.torsions,
                      type_params, root=int(inv[0]))
    tors = r.uniform(-math.pi, math.pi, lig.n_torsions)
    g = np.concatenate([[1.0, 2.0, 3.0], [0.4, 0.3, -0.2, 0.8], tors])
    x1 = OP.pose(lig, g)
    x2 = OP.pose(lig2, g)
    assert np.allclose(x1[perm], x2, atol=1e-12)
    e1, e2 = _intra(lig, x1), _intra(lig2, x2)
    assert abs(e1 - e2) <= 1e-12 * max(1.0, abs(e1))


@pytest.mark.parametrize("n,t,seed", [(20, 4, 51), (40, 8, 52)])
def test_intra_zero_net_force_and_torque(n, t, seed, type_params):
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    g = np.concatenate([r.normal(size=3), r.normal(size=4), r.uniform(-math.pi, math.pi, lig.n_torsions)])
    x = OP.pose(lig, g)
    F = np.zeros_like(x)
    scale = 0.0
    for (i, j) in lig.pairs:
        d = x[i] - x[j]
        rr = np.linalg.norm(d)
        dedr = S.pair_energy(rr, *S.pair_params(lig, i, j))[1]
        F[i] += dedr * d / rr
        F[j] -= dedr * d / rr
        scale += abs(dedr)
    assert np.all(np.abs(F.sum(axis=0)) <= 1e-12 * max(1.0, scale))
    assert np.all(np.abs(np.cross(x - g[0:3], F).sum(axis=0)) <= 1e-11 * max(1.0, scale))


def test_single_atom_energy_is_map_interpolation(type_params):
    g = _grid(12, 8)
    lig = OL.prepare(np.array([[0.3, -0.2, 0.1]]), [4], [0.25], np.zeros((0, 2), int),
                     np.zeros(0, int), type_params)
    p = np.array([0.2, -0.4, 0.35])
    genes = np.concatenate([p, [0.1, 0.7, 0.2, -0.3]])
    res = S.energy_and_gradient(g, lig, genes)
    gp = (p - g.origin) / g.spacing
    want = (S.trilinear(g.maps[4], gp)[0] + 0.25 * S.trilinear(g.maps[7], gp)[0]
            + 0.25 * S.trilinear(g.maps[8], gp)[0])
    assert abs(res.energy - want) < 1e-12
    assert np.allclose(res.grad[3:7], 0.0, atol=1e-12)


# ------------------------------------------------------------------ gradient
def _fd_grad(g, lig, genes, h=1e-6):
    out = np.zeros_like(genes)
    for k in range(genes.size):
        e = np.zeros_like(genes)
        e[k] = h
        out[k] = (S.energy(g, lig, genes + e) - S.energy(g, lig, genes - e)) / (2 * h)
    return out


@pytest.mark.parametrize("n,t,seed,npose", [(20, 4, 61, 40), (40, 8, 62, 20), (12, 9, 63, 20)])
def test_gradient_matches_finite_differences(n, t, seed, npose, type_params):
    g = _grid(40, 9)
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    checked = 0
    for _ in range(npose * 3):
        genes = np.concatenate([r.uniform(-3, 3, 3), r.normal(size=4),
                                r.uniform(-math.pi, math.pi, lig.n_torsions)])
        res = S.energy_and_gradient(g, lig, genes)
        if res.margin < 1e-3:
            continue   # within reach of a kink of the piecewise-smooth energy
        fd = _fd_grad(g, lig, genes)
        err = np.abs(fd - res.grad)
        # analytic error budget + the finite difference's own rounding noise (~eps*|E|/h)
        fd_noise = 10.0 * np.finfo(float).eps * res.scale_energy / 1e-6
        assert np.all(err <= 1e-6 * np.maximum(np.abs(res.grad), res.scale_grad) + fd_noise), (err, res.grad)
        checked += 1
        if checked == npose:
            break
    assert checked == npose


def test_quaternion_gradient_tangent_and_scale(type_params):
    g = _grid(40, 10)
    lig = _lig(20, 4, 71, type_params)
    r = np.random.default_rng(71)
    for _ in range(10):
        genes = np.concatenate([r.uniform(-2, 2, 3), r.normal(size=4), r.uniform(-3, 3, 4)])
        res = S.energy_and_gradient(g, lig, genes)
        q = genes[3:7]
        assert abs(q @ res.grad[3:7]) <= 1e-10 * max(1.0, res.scale_grad[3])
        g2 = genes.copy()
        g2[3:7] *= 2.5
        res2 = S.energy_and_gradient(g, lig, g2)
        assert abs(res2.energy - res.energy) <= 1e-12 * max(1.0, abs(res.energy))
        assert np.allclose(res2.grad[3:7] * 2.5, res.grad[3:7], atol=1e-9 * max(1.0, res.scale_grad[3]))


def _dR_dq(q):
    """Derivative of R(q/|q|) with respect to each raw component q_j, by differentiating the
    matrix entries (product rule through the normalisation)."""
    qn = np.linalg.norm(q)
    u = q / qn
    w, x, y, z = u
    # d R / d u_j for the entries of the unit-quaternion matrix
    dRu = np.array([
        [[0, -2 * z, 2 * y], [2 * z, 0, -2 * x], [-2 * y, 2 * x, 0]],
        [[0, 2 * y, 2 * z], [2 * y, -4 * x, -2 * w], [2 * z, 2 * w, -4 * x]],
        [[-4 * y, 2 * x, 2 * w], [2 * x, 0, 2 * z], [-2 * w, 2 * z, -4 * y]],
        [[-4 * z, -2 * w, 2 * x], [2 * w, -4 * z, 2 * y], [2 * x, 2 * y, 0]],
    ])
    J = (np.eye(4) - np.outer(u, u)) / qn     # d u / d q
    return np.einsum("jab,jk->kab", dRu, J)


def test_quaternion_gradient_via_matrix_chain_rule(type_params):
    g = _grid(40, 11)
    lig = _lig(20, 4, 81, type_params)
    r = np.random.default_rng(81)
    for _ in range(10):
        genes = np.concatenate([r.uniform(-2, 2, 3), r.normal(size=4), r.uniform(-3, 3, 4)])
        res = S.energy_and_gradient(g, lig, genes)
        p = OP.internal_coords(lig, genes)
        dR = _dR_dq(genes[3:7])
        want = np.array([np.sum(res.forces * (p @ dR[k].T)) for k in range(4)])
        assert np.allclose(want, res.grad[3:7], rtol=1e-9, atol=1e-9 * max(1.0, res.scale_grad[3]))


def test_gradient_translation_is_net_force(type_params):
    g = _grid(40, 12)
    lig = _lig(20, 4, 91, type_params)
    genes = np.concatenate([[0.5, -0.5, 1.0], [1, 0, 0, 0], np.zeros(4)])
    res = S.energy_and_gradient(g, lig, genes)
    assert np.allclose(res.grad[0:3], res.forces.sum(axis=0))
