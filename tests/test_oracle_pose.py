"""Pins of the oracle's genotype -> pose construction."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import ligand as OL
from oracle import pose as OP
from workload import synth


def _rand_quats(n, seed):
    r = np.random.default_rng(seed)
    q = r.normal(size=(n, 4))
    return q


def test_quat_matrix_orthonormal_det1():
    for q in _rand_quats(50, 1):
        R = OP.quat_to_matrix(q)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13


def test_quat_matrix_matches_scipy():
    for q in _rand_quats(50, 2):
        w, x, y, z = q / np.linalg.norm(q)
        ref = Rotation.from_quat([x, y, z, w]).as_matrix()     # scipy order: x, y, z, w
        assert np.allclose(OP.quat_to_matrix(q), ref, atol=1e-13)


def test_quat_scale_invariance_and_product():
    qs = _rand_quats(20, 3)
    for a, b in zip(qs[:10], qs[10:]):
        assert np.allclose(OP.quat_to_matrix(3.7 * a), OP.quat_to_matrix(a), atol=1e-13)
        assert np.allclose(OP.quat_to_matrix(-a), OP.quat_to_matrix(a), atol=1e-13)
        ab = OP.quat_mul(a / np.linalg.norm(a), b / np.linalg.norm(b))
        assert np.allclose(OP.quat_to_matrix(ab), OP.quat_to_matrix(a) @ OP.quat_to_matrix(b),
                           atol=1e-12)


def test_rodrigues_matches_scipy_rotvec():
    r = np.random.default_rng(4)
    for _ in range(30):
        u = r.normal(size=3)
        u /= np.linalg.norm(u)
        th = r.uniform(-math.pi, math.pi)
        v = r.normal(size=(5, 3))
        ref = Rotation.from_rotvec(th * u).apply(v)
        assert np.allclose(OP.rodrigues(u, th, v), ref, atol=1e-13)


def _dihedral(p0, p1, p2, p3):
    b0, b1, b2 = p0 - p1, p2 - p1, p3 - p2
    b1n = b1 / np.linalg.norm(b1)
    v = b0 - (b0 @ b1n) * b1n
    w = b2 - (b2 @ b1n) * b1n
    return math.atan2(np.cross(b1n, v) @ w, v @ w)


def _lig(n, t, seed, tp):
    return OL.from_synth(synth.make_ligand(n, t, seed, tp))


@pytest.mark.parametrize("n,t,seed", [(12, 4, 1), (20, 4, 2), (40, 8, 3), (30, 20, 4)])
def test_torsion_changes_its_dihedral_by_theta(n, t, seed, type_params):
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    genes = np.zeros(lig.n_genes)
    genes[3] = 1.0
    genes[7:] = r.uniform(-math.pi, math.pi, lig.n_torsions)
    x0 = lig.p0
    x1 = OP.pose(lig, genes)
    for k in range(lig.n_torsions):
        a, b = lig.tors_a[k], lig.tors_b[k]
        c = next(i for i in lig.neighbours[a] if i != b)
        d = next(i for i in lig.neighbours[b] if i != a)
        d0 = _dihedral(x0[c], x0[a], x0[b], x0[d])
        d1 = _dihedral(x1[c], x1[a], x1[b], x1[d])
        diff = OP.wrap_angle(d1 - d0 - genes[7 + k])
        assert abs(diff) < 1e-10, (k, diff)


@pytest.mark.parametrize("n,t,seed", [(20, 4, 5), (40, 8, 6), (60, 25, 7)])
def test_bond_geometry_preserved(n, t, seed, type_params):
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    genes = np.concatenate([r.normal(size=3), r.normal(size=4),
                            r.uniform(-math.pi, math.pi, lig.n_torsions)])
    x = OP.pose(lig, genes)
    for a in range(lig.n_atoms):
        for b in lig.neighbours[a]:
            assert abs(np.linalg.norm(x[a] - x[b]) - np.linalg.norm(lig.p0[a] - lig.p0[b])) < 1e-12
            for c in lig.neighbours[b]:
                if c != a:   # 1-3 distances fix the bond angles
                    assert abs(np.linalg.norm(x[a] - x[c]) - np.linalg.norm(lig.p0[a] - lig.p0[c])) < 1e-12


def _leaf_to_root(lig, genes):
    """Independent construction: deepest torsion first, each about its reference-frame axis."""
    p = lig.p0.copy()
    order = sorted(range(lig.n_torsions), key=lambda k: -lig.depth[lig.tors_a[k]])
    for k in order:
        a, b = lig.tors_a[k], lig.tors_b[k]
        u = lig.p0[b] - lig.p0[a]
        u /= np.linalg.norm(u)
        th = genes[7 + k]
        m = lig.moving[k]
        v = p[m] - lig.p0[a]
        c, s = math.cos(th), math.sin(th)
        p[m] = lig.p0[a] + v * c + np.cross(u, v) * s + np.outer(v @ u, u) * (1 - c)
    w, x, y, z = genes[3:7] / np.linalg.norm(genes[3:7])
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    return p @ R.T + genes[0:3]


@pytest.mark.parametrize("n,t,seed", [(20, 4, 8), (40, 8, 9), (90, 32, 10)])
def test_root_to_leaf_equals_leaf_to_root(n, t, seed, type_params):
    lig = _lig(n, t, seed, type_params)
    r = np.random.default_rng(seed)
    for _ in range(5):
        genes = np.concatenate([r.normal(size=3) * 5, r.normal(size=4),
                                r.uniform(-math.pi, math.pi, lig.n_torsions)])
        assert np.allclose(OP.pose(lig, genes), _leaf_to_root(lig, genes), atol=1e-12)


def test_rigid_pose_and_centroid(type_params):
    lig = _lig(20, 4, 11, type_params)
    assert np.allclose(lig.p0.mean(axis=0), 0.0, atol=1e-12)
    genes = np.zeros(lig.n_genes)
    genes[0:3] = [1.0, -2.0, 3.0]
    genes[3:7] = [0.3, 0.1, -0.5, 0.8]
    x = OP.pose(lig, genes)
    assert np.allclose(x, lig.p0 @ OP.quat_to_matrix(genes[3:7]).T + genes[0:3], atol=1e-13)
    assert np.allclose(x.mean(axis=0), genes[0:3], atol=1e-12)


def test_wrap_angle():
    for th, want in [(0.0, 0.0), (math.pi, math.pi), (-math.pi, math.pi), (3 * math.pi, math.pi),
                     (math.pi + 0.1, -math.pi + 0.1), (-math.pi - 0.1, math.pi - 0.1), (7.0, 7.0 - 2 * math.pi)]:
        assert abs(OP.wrap_angle(th) - want) < 1e-12


def test_ligand_validation(type_params):
    lig = synth.make_ligand(10, 3, 12, type_params)
    with pytest.raises(OL.LigandError):
        OL.prepare(lig.xyz, lig.types, lig.charges, lig.bonds[:-1], lig.torsions, type_params)
    bad_types = lig.types.copy()
    bad_types[0] = 9
    with pytest.raises(OL.LigandError):
        OL.prepare(lig.xyz, bad_types, lig.charges, lig.bonds, lig.torsions, type_params)
    # a terminal bond (one end has degree 1) cannot be a torsion
    deg = np.bincount(lig.bonds.ravel(), minlength=10)
    term = [i for i, (a, b) in enumerate(lig.bonds) if deg[a] == 1 or deg[b] == 1]
    with pytest.raises(OL.LigandError):
        OL.prepare(lig.xyz, lig.types, lig.charges, lig.bonds, np.array([term[0]]), type_params)
