"""Energy and analytic genotype gradient of one pose (oracle, FP64).

The score has the two parts the paper names (Background, "Design and Structure of
MiniMDock"): the interaction of every ligand atom with the receptor's precomputed
3-D grid, and self-interactions among ligand atoms (hydrogen bonding, van der
Waals, desolvation; electrostatics added as in the AutoDock4 lineage).  The
per-atom energies are summed into one value per pose (Section "Approach 1",
listing of decomposed target functions).  Forms and constants: `constants`.

Grid part, per atom i at grid coordinate g = (x_i - o)/h:
  inside (0 <= g_a < n_a - 1 on every axis): trilinear interpolation of the atom's
  type map, plus q_i times the electrostatic map, plus |q_i| times the desolvation
  map, and the exact derivative of that interpolant;
  outside: P_OUT + K_OUT * d^2 with d the distance to the grid box, gradient
  2 K_OUT (x - clamp(x)).
Pair part, per listed pair at distance r (r~ = max(r, R_MIN), gradient 0 below
R_MIN): 12-6 vdW, or 12-10 H-bond for donor/acceptor pairs (no angular term),
within CUTOFF; Coulomb with eps(r) within CUTOFF_EL; Gaussian desolvation within
CUTOFF.

Genotype gradient from the per-atom forces F_i = dE/dx_i:
  dE/dt       = sum_i F_i
  torque      tau = sum_i (x_i - t) x F_i
  dE/dq       = (-2 tau.v, 2 (w tau - v x tau)) / |q|   for q/|q| = (w, v)
  dE/dtheta_k = u_k . sum_{i moved by k} (x_i - x_{a_k}) x F_i, u_k the posed axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import constants as C
from .pose import pose


@dataclass
class Grid:
    maps: np.ndarray       # float64 [9][nz][ny][nx]
    origin: np.ndarray     # [3]
    spacing: float

    @property
    def n_xyz(self):
        nz, ny, nx = self.maps.shape[1:]
        return np.array([nx, ny, nz])


def make_grid(maps, origin, spacing) -> Grid:
    return Grid(maps=np.asarray(maps, dtype=np.float64), origin=np.asarray(origin, np.float64),
                spacing=float(spacing))


# ---------------------------------------------------------------- grid term
def trilinear(vol, g):
    """Value and d/dg of the trilinear interpolant of vol[z][y][x] at grid point g=(gx,gy,gz),
    which must satisfy 0 <= g_a < n_a - 1."""
    i = np.floor(g).astype(np.int64)
    f = g - i
    val = 0.0
    dval = np.zeros(3)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                m = vol[i[2] + cz, i[1] + cy, i[0] + cx]
                wx = f[0] if cx else 1.0 - f[0]
                wy = f[1] if cy else 1.0 - f[1]
                wz = f[2] if cz else 1.0 - f[2]
                val += wx * wy * wz * m
                sx = 1.0 if cx else -1.0
                sy = 1.0 if cy else -1.0
                sz = 1.0 if cz else -1.0
                dval += m * np.array([sx * wy * wz, wx * sy * wz, wx * wy * sz])
    return val, dval


def inside(grid: Grid, x):
    g = (np.asarray(x, np.float64) - grid.origin) / grid.spacing
    return bool(np.all(g >= 0.0) and np.all(g < grid.n_xyz - 1)), g


def atom_grid_energy(grid: Grid, x, atype, charge):
    """Energy and dE/dx of one atom against the receptor maps; also the sum of the
    absolute values of the three map contributions (a conditioning scale)."""
    ins, g = inside(grid, x)
    if ins:
        vt, dt = trilinear(grid.maps[atype], g)
        ve, de = trilinear(grid.maps[C.N_TYPES], g)
        vd, dd = trilinear(grid.maps[C.N_TYPES + 1], g)
        aq = abs(charge)
        e = vt + charge * ve + aq * vd
        de_dx = (dt + charge * de + aq * dd) / grid.spacing
        scale = abs(vt) + abs(charge * ve) + abs(aq * vd)
        return e, de_dx, scale
    lo = grid.origin
    hi = grid.origin + (grid.n_xyz - 1) * grid.spacing
    xc = np.clip(x, lo, hi)
    d = np.asarray(x) - xc
    e = C.P_OUT + C.K_OUT * float(d @ d)
    return e, 2.0 * C.K_OUT * d, abs(e)


# ---------------------------------------------------------------- pair terms
def dielectric(r):
    """Mehler-Solmajer eps(r) and d eps/dr."""
    ex = math.exp(-C.DIEL_LAMBDA * C.DIEL_B * r)
    den = 1.0 + C.DIEL_K * ex
    eps = C.DIEL_A + C.DIEL_B / den
    deps = C.DIEL_B * C.DIEL_K * C.DIEL_LAMBDA * C.DIEL_B * ex / (den * den)
    return eps, deps


def pair_params(lig, i, j):
    """Coefficients of one pair: (is_hb, C12, Cn, qq, ds) where Cn is C6 or C10."""
    tp = lig.type_params
    ti, tj = lig.types[i], lig.types[j]
    role_i, role_j = int(tp[ti, 4]), int(tp[tj, 4])
    acc = None
    if role_i == C.HB_DONOR and role_j == C.HB_ACCEPTOR:
        acc = tj
    elif role_i == C.HB_ACCEPTOR and role_j == C.HB_DONOR:
        acc = ti
    if acc is not None:
        r_hb, e_hb = tp[acc, 5], tp[acc, 6]
        c12 = 5.0 * e_hb * r_hb ** 12
        cn = 6.0 * e_hb * r_hb ** 10
        is_hb = True
    else:
        rij = 0.5 * (tp[ti, 0] + tp[tj, 0])
        eij = math.sqrt(tp[ti, 1] * tp[tj, 1])
        c12 = eij * rij ** 12
        cn = 2.0 * eij * rij ** 6
        is_hb = False
    qi, qj = lig.charges[i], lig.charges[j]
    si = tp[ti, 3] + C.QASP * abs(qi)
    sj = tp[tj, 3] + C.QASP * abs(qj)
    ds = si * tp[tj, 2] + sj * tp[ti, 2]
    return is_hb, c12, cn, qi * qj, ds


def pair_energy(r, is_hb, c12, cn, qq, ds):
    """Pair energy at distance r, its derivative de/dr, and the sum of |term| values.
    Returns the three terms separately as well: (e, dedr, scale, (e_vdw_hb, e_el, e_ds))."""
    rt = max(r, C.R_MIN)
    clamped = r < C.R_MIN
    e_lj = e_el = e_ds = 0.0
    d_lj = d_el = d_ds = 0.0
    if r < C.CUTOFF:
        if is_hb:
            e_lj = C.W_HB * (c12 / rt ** 12 - cn / rt ** 10)
            d_lj = C.W_HB * (-12.0 * c12 / rt ** 13 + 10.0 * cn / rt ** 11)
        else:
            e_lj = C.W_VDW * (c12 / rt ** 12 - cn / rt ** 6)
            d_lj = C.W_VDW * (-12.0 * c12 / rt ** 13 + 6.0 * cn / rt ** 7)
        gauss = math.exp(-rt * rt / (2.0 * C.DESOLV_SIGMA ** 2))
        e_ds = C.W_DS * ds * gauss
        d_ds = -rt / C.DESOLV_SIGMA ** 2 * e_ds
    if r < C.CUTOFF_EL:
        eps, deps = dielectric(rt)
        e_el = C.W_EL * C.COULOMB * qq / (rt * eps)
        d_el = -C.W_EL * C.COULOMB * qq * (eps + rt * deps) / (rt * eps) ** 2
    e = e_lj + e_el + e_ds
    dedr = 0.0 if clamped else d_lj + d_el + d_ds
    scale = abs(e_lj) + abs(e_el) + abs(e_ds)
    return e, dedr, scale, (e_lj, e_el, e_ds)


# ---------------------------------------------------------------- whole pose
@dataclass
class EvalResult:
    energy: float
    grad: np.ndarray          # [G]
    x: np.ndarray             # posed coordinates [N][3]
    forces: np.ndarray        # dE/dx_i [N][3]
    e_inter: float
    e_intra: float
    scale_energy: float       # sum of |every atom term and pair term|
    scale_grad: np.ndarray    # [G] sum of |contributions| to each gene's gradient
    margin: float             # distance (grid units / Angstrom) to the nearest kink


def energy_and_gradient(grid: Grid, lig, genes, want_margin=True) -> EvalResult:
    genes = np.asarray(genes, dtype=np.float64)
    n = lig.n_atoms
    x = pose(lig, genes)
    F = np.zeros((n, 3))
    Fabs = np.zeros((n, 3))
    e_inter = e_intra = 0.0
    scale = 0.0
    margin = math.inf
    # grid part
    for i in range(n):
        e, dedx, s = atom_grid_energy(grid, x[i], lig.types[i], lig.charges[i])
        e_inter += e
        scale += s
        F[i] += dedx
        Fabs[i] += np.abs(dedx)
        if want_margin:
            ins, g = inside(grid, x[i])
            margin = min(margin, float(np.min(np.abs(g))),
                         float(np.min(np.abs(g - (grid.n_xyz - 1)))))
            if ins:
                frac = g - np.floor(g)
                margin = min(margin, float(np.min(np.minimum(frac, 1.0 - frac))))
    # pair part
    for (i, j) in lig.pairs:
        d = x[i] - x[j]
        r = float(np.sqrt(d @ d))
        is_hb, c12, cn, qq, ds = pair_params(lig, i, j)
        e, dedr, s, _ = pair_energy(r, is_hb, c12, cn, qq, ds)
        e_intra += e
        scale += s
        if dedr != 0.0:
            f = dedr * d / r
            F[i] += f
            F[j] -= f
            Fabs[i] += np.abs(f)
            Fabs[j] += np.abs(f)
        if want_margin:
            margin = min(margin, abs(r - C.R_MIN), abs(r - C.CUTOFF), abs(r - C.CUTOFF_EL))

    G = lig.n_genes
    grad = np.zeros(G)
    sgrad = np.zeros(G)
    t = genes[0:3]
    grad[0:3] = F.sum(axis=0)
    sgrad[0:3] = Fabs.sum(axis=0)
    qn = np.linalg.norm(genes[3:7])
    w = genes[3] / qn
    v = genes[4:7] / qn
    rel = x - t
    tau = np.cross(rel, F).sum(axis=0)
    grad[3] = -2.0 * (tau @ v) / qn
    grad[4:7] = 2.0 * (w * tau - np.cross(v, tau)) / qn
    sgrad[3:7] = 2.0 * float(np.sum(np.linalg.norm(rel, axis=1) * np.linalg.norm(Fabs, axis=1))) / qn
    for k in range(lig.n_torsions):
        a, b = lig.tors_a[k], lig.tors_b[k]
        u = x[b] - x[a]
        u = u / np.linalg.norm(u)
        m = lig.moving[k]
        arm = x[m] - x[a]
        grad[7 + k] = float(u @ np.cross(arm, F[m]).sum(axis=0))
        sgrad[7 + k] = float(np.sum(np.linalg.norm(arm, axis=1) * np.linalg.norm(Fabs[m], axis=1)))
    return EvalResult(energy=e_inter + e_intra, grad=grad, x=x, forces=F, e_inter=e_inter,
                      e_intra=e_intra, scale_energy=scale, scale_grad=sgrad, margin=margin)


def energy(grid: Grid, lig, genes) -> float:
    return energy_and_gradient(grid, lig, genes, want_margin=False).energy
