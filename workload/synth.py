"""Seeded synthetic docking inputs: receptor grid maps, an atom-type table and ligands.

This module only draws inputs.  It holds none of the docking method's arithmetic
(no pose construction, no scoring, no search); the oracle and the HIP library both
receive what it produces as plain arrays.

Workload shapes follow the paper's description of the problem (Background,
"Design and Structure of MiniMDock"): a receptor represented as a 3-D grid of
precomputed interaction values, a ligand of point atoms joined by a bond tree whose
rotatable bonds (together with the rigid-body translation and orientation) are the
degrees of freedom, and inputs that differ by atom and rotatable-bond counts.
The paper's own ligands and receptor are not available, so every input here is
synthetic:

* Maps: each of the 9 maps (7 atom-type affinity maps, 1 electrostatic map,
  1 desolvation map) is a sum of 30 random 3-D Gaussians (centres uniform in the
  box, width U[1.5, 4.0] Angstrom, amplitude U[-6, +14] kcal/mol), clipped to
  [-2, +10], stored as float32 with layout [map][z][y][x].
* Atom types: 7 types with radius R in [2.0, 4.2] A, well depth eps in
  [0.02, 0.25] kcal/mol, atomic volume in [0, 35] A^3, solvation parameter in
  [-0.003, 0.001]; types 3 and 4 are hydrogen-bond acceptors (R_hb in [1.8, 2.0] A,
  eps_hb in [1, 5] kcal/mol), type 6 is the donor.
* Ligand: a random tree of heavy atoms (1.5 A bonds, 109.5 degree angles, random
  dihedrals, non-bonded contacts kept >= 2.0 A), a backbone path long enough to hold
  the requested rotatable bonds, types uniform over the 7 types, charges U[-0.5, 0.5]
  with the mean removed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_TYPES = 7
N_MAPS = N_TYPES + 2          # type maps, then electrostatic, then desolvation
HB_NONE, HB_DONOR, HB_ACCEPTOR = 0, 1, 2


@dataclass
class Receptor:
    """Grid maps plus grid geometry.  maps: float32 [N_MAPS][nz][ny][nx]."""
    maps: np.ndarray
    spacing: float
    origin: np.ndarray          # float64 [3], position of node (0,0,0) in Angstrom

    @property
    def shape_xyz(self):
        nz, ny, nx = self.maps.shape[1:]
        return (nx, ny, nz)


@dataclass
class Ligand:
    """A ligand as the library's ligand descriptor takes it (all arrays plain numpy)."""
    xyz: np.ndarray             # float32 [n_atoms][3] reference conformation
    types: np.ndarray           # int32 [n_atoms]
    charges: np.ndarray         # float32 [n_atoms]
    bonds: np.ndarray           # int32 [n_bonds][2], connected (the generated ligands are trees)
    torsions: np.ndarray        # int32 [n_torsions], indices into bonds
    root: int = 0
    type_params: np.ndarray = field(default=None)   # float32 [N_TYPES][7]

    @property
    def n_atoms(self):
        return int(self.xyz.shape[0])

    @property
    def n_torsions(self):
        return int(self.torsions.shape[0])

    @property
    def n_genes(self):
        return 7 + self.n_torsions


def make_type_params(seed: int) -> np.ndarray:
    """float32 [7][7] columns: R_eq, eps, vol, solpar, hb_role, R_hb, eps_hb."""
    rng = np.random.default_rng([seed, 0x7A9E])
    tp = np.zeros((N_TYPES, 7), dtype=np.float64)
    tp[:, 0] = rng.uniform(2.0, 4.2, N_TYPES)
    tp[:, 1] = rng.uniform(0.02, 0.25, N_TYPES)
    tp[:, 2] = rng.uniform(0.0, 35.0, N_TYPES)
    tp[:, 3] = rng.uniform(-0.003, 0.001, N_TYPES)
    for t in range(N_TYPES):
        if t in (3, 4):
            tp[t, 4] = HB_ACCEPTOR
            tp[t, 5] = rng.uniform(1.8, 2.0)
            tp[t, 6] = rng.uniform(1.0, 5.0)
        elif t == 6:
            tp[t, 4] = HB_DONOR
    return tp.astype(np.float32)


def make_receptor(n: int, seed: int, spacing: float = 0.375, n_gauss: int = 30,
                  clip=(-2.0, 10.0)) -> Receptor:
    """n^3 grid centred on the origin; per-map seeds derived from `seed`."""
    origin = np.full(3, -0.5 * (n - 1) * spacing, dtype=np.float64)
    ax = origin[0] + spacing * np.arange(n, dtype=np.float64)
    lo, hi = ax[0], ax[-1]
    maps = np.empty((N_MAPS, n, n, n), dtype=np.float32)
    for m in range(N_MAPS):
        rng = np.random.default_rng([seed, 0x3A95, m])
        acc = np.zeros((n, n, n), dtype=np.float64)
        for _ in range(n_gauss):
            c = rng.uniform(lo, hi, 3)
            s = rng.uniform(1.5, 4.0)
            a = rng.uniform(-6.0, 14.0)
            gx = np.exp(-((ax - c[0]) ** 2) / (2 * s * s))
            gy = np.exp(-((ax - c[1]) ** 2) / (2 * s * s))
            gz = np.exp(-((ax - c[2]) ** 2) / (2 * s * s))
            acc += a * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        maps[m] = np.clip(acc, clip[0], clip[1]).astype(np.float32)
    return Receptor(maps=maps, spacing=float(spacing), origin=origin)


def _place(p_par, p_gp, p_ref, bond, angle, dihedral):
    """Internal-coordinate placement of a new atom bonded to p_par."""
    b = p_par - p_gp
    b /= np.linalg.norm(b)
    r = p_gp - p_ref
    n = np.cross(r, b)
    if np.linalg.norm(n) < 1e-6:
        n = np.cross(b, np.array([1.0, 0.0, 0.0]))
        if np.linalg.norm(n) < 1e-6:
            n = np.cross(b, np.array([0.0, 1.0, 0.0]))
    n /= np.linalg.norm(n)
    m = np.cross(n, b)
    d = np.array([-bond * math.cos(angle),
                  bond * math.sin(angle) * math.cos(dihedral),
                  bond * math.sin(angle) * math.sin(dihedral)])
    return p_par + d[0] * b + d[1] * m + d[2] * n


def make_ligand(n_atoms: int, n_torsions: int, seed: int, type_params: np.ndarray,
                bond_len: float = 1.5, min_contact: float = 2.0,
                max_valence: int = 3) -> Ligand:
    """Random heavy-atom tree with a backbone of n_torsions+3 atoms.

    The number of rotatable bonds is capped at min(n_torsions, n_atoms-3, 32): a tree
    has at most n_atoms-3 bonds whose both ends carry further atoms, and rotating a
    terminal bond moves nothing.
    """
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    n_tors = max(0, min(int(n_torsions), n_atoms - 3, 32))
    angle = math.radians(109.5)
    for attempt in range(200):
        rng = np.random.default_rng([seed, 0x11A6, attempt])
        pos = np.zeros((n_atoms, 3))
        parent = -np.ones(n_atoms, dtype=np.int64)
        deg = np.zeros(n_atoms, dtype=np.int64)
        nb = [[] for _ in range(n_atoms)]
        ok = True
        backbone = min(n_atoms, n_tors + 3) if n_tors > 0 else min(n_atoms, 3)
        for k in range(1, n_atoms):
            placed = False
            for _try in range(60):
                if k < backbone:
                    par = k - 1
                else:
                    cand = [a for a in range(k) if deg[a] < max_valence]
                    if not cand:
                        break
                    par = int(cand[rng.integers(len(cand))])
                if par == 0 and k == 1:
                    p = pos[0] + np.array([bond_len, 0.0, 0.0])
                else:
                    gp = parent[par] if parent[par] >= 0 else (nb[par][0] if nb[par] else -1)
                    if gp < 0:
                        p = pos[par] + bond_len * _unit(rng.normal(size=3))
                    else:
                        ref_c = [a for a in nb[gp] if a != par]
                        if parent[gp] >= 0:
                            ref_c.append(int(parent[gp]))
                        if ref_c:
                            ref = pos[ref_c[0]]
                        else:
                            ref = pos[gp] + _unit(rng.normal(size=3))
                        p = _place(pos[par], pos[gp], ref, bond_len, angle,
                                   rng.uniform(0.0, 2.0 * math.pi))
                d = np.linalg.norm(pos[:k] - p, axis=1)
                d[par] = np.inf
                if parent[par] >= 0:
                    d[parent[par]] = np.inf   # 1-3 neighbour via the parent's parent
                for a in nb[par]:
                    d[a] = np.inf             # 1-3 neighbours via siblings
                if d.min() >= min_contact:
                    pos[k] = p
                    parent[k] = par
                    deg[k] += 1
                    deg[par] += 1
                    nb[k].append(par)
                    nb[par].append(k)
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if not ok:
            continue
        bonds = np.array([[parent[k], k] for k in range(1, n_atoms)], dtype=np.int32).reshape(-1, 2)
        internal = [bi for bi, (a, b) in enumerate(bonds) if deg[a] >= 2 and deg[b] >= 2]
        if len(internal) < n_tors:
            continue
        tors = np.sort(rng.choice(internal, size=n_tors, replace=False)).astype(np.int32) \
            if n_tors > 0 else np.zeros(0, dtype=np.int32)
        types = rng.integers(0, N_TYPES, n_atoms).astype(np.int32)
        q = rng.uniform(-0.5, 0.5, n_atoms)
        q -= q.mean()
        # shuffle bond order and bond direction so consumers cannot rely on generation order
        perm = rng.permutation(bonds.shape[0])
        bonds = bonds[perm]
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        tors = np.sort(inv[tors]).astype(np.int32) if n_tors > 0 else tors
        flip = rng.integers(0, 2, bonds.shape[0]).astype(bool)
        bonds[flip] = bonds[flip][:, ::-1]
        return Ligand(xyz=pos.astype(np.float32), types=types, charges=q.astype(np.float32),
                      bonds=np.ascontiguousarray(bonds, dtype=np.int32),
                      torsions=np.ascontiguousarray(tors, dtype=np.int32),
                      root=0, type_params=np.asarray(type_params, dtype=np.float32))
    raise RuntimeError(f"could not build a ligand with {n_atoms} atoms / {n_tors} torsions")


def _unit(v):
    return v / np.linalg.norm(v)


def random_genes(lig: Ligand, rec: Receptor, n_poses: int, seed: int,
                 margin: float = 0.0) -> np.ndarray:
    """Random genotypes [n_poses][7+T] (float32): translation uniform in the grid box
    shrunk by `margin` Angstrom, a uniformly random unit quaternion (w, x, y, z),
    torsion angles uniform in (-pi, pi]."""
    rng = np.random.default_rng([seed, 0x6E9E])
    nx, ny, nz = rec.shape_xyz
    ext = np.array([nx - 1, ny - 1, nz - 1], dtype=np.float64) * rec.spacing
    lo = rec.origin + margin
    hi = rec.origin + ext - margin
    g = np.zeros((n_poses, lig.n_genes), dtype=np.float64)
    g[:, 0:3] = rng.uniform(lo, hi, (n_poses, 3))
    q = rng.normal(size=(n_poses, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    g[:, 3:7] = q
    g[:, 7:] = rng.uniform(-math.pi, math.pi, (n_poses, lig.n_torsions))
    return g.astype(np.float32)
