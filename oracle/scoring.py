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
    """Value and d/dg of the trilinear interpolant of vol[z][y][x] at grid point(s) g=(gx,gy,gz)
    (shape [3] or [M][3]), each satisfying 0 <= g_a < n_a - 1."""
    g = np.asarray(g, dtype=np.float64)
    single = g.ndim == 1
    g = g.reshape(-1, 3)
    i = np.floor(g).astype(np.int64)
    f = g - i
    val = np.zeros(g.shape[0])
    dval = np.zeros_like(g)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                m = vol[i[:, 2] + cz, i[:, 1] + cy, i[:, 0] + cx]
                wx = f[:, 0] if cx else 1.0 - f[:, 0]
                wy = f[:, 1] if cy else 1.0 - f[:, 1]
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                val += wx * wy * wz * m
                sx = 1.0 if cx else -1.0
                sy = 1.0 if cy else -1.0
                sz = 1.0 if cz else -1.0
                dval += m[:, None] * np.stack([sx * wy * wz, wx * sy * wz, wx * wy * sz], axis=1)
    if single:
        return float(val[0]), dval[0]
    return val, dval


def trilinear_abs(vol, g):
    """Condition scales of the interpolant at g ([M][3]): sum_c w_c |m_c| and, per axis,
    sum_c |m_c| |d w_c / d g_a| -- the sums of the absolute values of the terms that make up
    the value and its derivative."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, 3)
    i = np.floor(g).astype(np.int64)
    f = g - i
    sval = np.zeros(g.shape[0])
    sder = np.zeros_like(g)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                m = np.abs(vol[i[:, 2] + cz, i[:, 1] + cy, i[:, 0] + cx])
                wx = f[:, 0] if cx else 1.0 - f[:, 0]
                wy = f[:, 1] if cy else 1.0 - f[:, 1]
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                sval += wx * wy * wz * m
                sder += m[:, None] * np.stack([wy * wz, wx * wz, wx * wy], axis=1)
    return sval, sder


def inside(grid: Grid, x):
    """Whether point(s) x lie inside the interpolation box, and their grid coordinates."""
    g = (np.asarray(x, np.float64) - grid.origin) / grid.spacing
    ins = np.all(g >= 0.0, axis=-1) & np.all(g < grid.n_xyz - 1, axis=-1)
    return (bool(ins) if np.ndim(ins) == 0 else ins), g


def grid_energies(grid: Grid, x, types, charges, with_force_scale=False):
    """Per-atom grid energies e_i [N], dE/dx_i [N][3] and |term| scales [N] for atoms x [N][3]
    (with_force_scale: also the per-component |term| scales of dE/dx_i, [N][3])."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    types = np.asarray(types).reshape(-1)
    q = np.asarray(charges, np.float64).reshape(-1)
    n = x.shape[0]
    e = np.zeros(n)
    de = np.zeros((n, 3))
    scale = np.zeros(n)
    fscale = np.zeros((n, 3))
    ins, g = inside(grid, x)
    ins = np.atleast_1d(ins)
    if np.any(ins):
        gi = g[ins]
        aq = np.abs(q[ins])
        vt = np.zeros(gi.shape[0])
        dt = np.zeros_like(gi)
        for t in np.unique(types[ins]):
            sel = types[ins] == t
            vt[sel], dt[sel] = trilinear(grid.maps[t], gi[sel])
        ve, dv_e = trilinear(grid.maps[C.N_TYPES], gi)
        vd, dv_d = trilinear(grid.maps[C.N_TYPES + 1], gi)
        e[ins] = vt + q[ins] * ve + aq * vd
        de[ins] = (dt + q[ins][:, None] * dv_e + aq[:, None] * dv_d) / grid.spacing
        st = np.zeros(gi.shape[0])
        sdt = np.zeros_like(gi)
        for t in np.unique(types[ins]):
            sel = types[ins] == t
            st[sel], sdt[sel] = trilinear_abs(grid.maps[t], gi[sel])
        se, sde = trilinear_abs(grid.maps[C.N_TYPES], gi)
        sd, sdd = trilinear_abs(grid.maps[C.N_TYPES + 1], gi)
        scale[ins] = st + aq * se + aq * sd
        fscale[ins] = (sdt + aq[:, None] * sde + aq[:, None] * sdd) / grid.spacing
    out = ~ins
    if np.any(out):
        lo = grid.origin
        hi = grid.origin + (grid.n_xyz - 1) * grid.spacing
        d = x[out] - np.clip(x[out], lo, hi)
        e[out] = C.P_OUT + C.K_OUT * np.sum(d * d, axis=1)
        de[out] = 2.0 * C.K_OUT * d
        scale[out] = np.abs(e[out])
        fscale[out] = np.abs(de[out])
    if with_force_scale:
        return e, de, scale, fscale
    return e, de, scale


def atom_grid_energy(grid: Grid, x, atype, charge):
    """Energy, dE/dx and |term| scale of one atom against the receptor maps."""
    e, de, s = grid_energies(grid, np.asarray(x, np.float64)[None, :], [atype], [charge])
    return float(e[0]), de[0], float(s[0])


# ---------------------------------------------------------------- pair terms
def dielectric(r):
    """Mehler-Solmajer eps(r) and d eps/dr."""
    ex = np.exp(-C.DIEL_LAMBDA * C.DIEL_B * np.asarray(r, np.float64))
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


def pair_table(lig):
    """pair_params of every listed pair as arrays (computed once per ligand)."""
    cached = getattr(lig, "_pair_table", None)
    if cached is None:
        rows = [pair_params(lig, i, j) for (i, j) in lig.pairs]
        if rows:
            cols = list(zip(*rows))
            cached = (np.array(cols[0], bool),) + tuple(np.array(c, np.float64) for c in cols[1:])
        else:
            cached = (np.zeros(0, bool),) + tuple(np.zeros(0) for _ in range(4))
        lig._pair_table = cached
    return cached


def pair_energy(r, is_hb, c12, cn, qq, ds):
    """Pair energy at distance(s) r, de/dr, the sum of |term| values, and the three terms
    (e_vdw_or_hb, e_el, e_ds).  Scalars or equal-length arrays."""
    scalar = np.ndim(r) == 0
    r = np.atleast_1d(np.asarray(r, np.float64))
    is_hb = np.broadcast_to(np.asarray(is_hb, bool), r.shape)
    c12, cn, qq, ds = (np.broadcast_to(np.asarray(a, np.float64), r.shape) for a in (c12, cn, qq, ds))
    rt = np.maximum(r, C.R_MIN)
    near = r < C.CUTOFF
    e_lj = np.where(is_hb, C.W_HB * (c12 / rt ** 12 - cn / rt ** 10),
                    C.W_VDW * (c12 / rt ** 12 - cn / rt ** 6))
    d_lj = np.where(is_hb, C.W_HB * (-12.0 * c12 / rt ** 13 + 10.0 * cn / rt ** 11),
                    C.W_VDW * (-12.0 * c12 / rt ** 13 + 6.0 * cn / rt ** 7))
    e_ds = C.W_DS * ds * np.exp(-rt * rt / (2.0 * C.DESOLV_SIGMA ** 2))
    d_ds = -rt / C.DESOLV_SIGMA ** 2 * e_ds
    e_lj, d_lj = np.where(near, e_lj, 0.0), np.where(near, d_lj, 0.0)
    e_ds, d_ds = np.where(near, e_ds, 0.0), np.where(near, d_ds, 0.0)
    eps, deps = dielectric(rt)
    e_el = C.W_EL * C.COULOMB * qq / (rt * eps)
    d_el = -C.W_EL * C.COULOMB * qq * (eps + rt * deps) / (rt * eps) ** 2
    far = r < C.CUTOFF_EL
    e_el, d_el = np.where(far, e_el, 0.0), np.where(far, d_el, 0.0)
    e = e_lj + e_el + e_ds
    dedr = np.where(r < C.R_MIN, 0.0, d_lj + d_el + d_ds)
    scale = np.abs(e_lj) + np.abs(e_el) + np.abs(e_ds)
    if scalar:
        return float(e[0]), float(dedr[0]), float(scale[0]), (float(e_lj[0]), float(e_el[0]), float(e_ds[0]))
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
    margin: float             # distance (grid units / Angstrom) to the nearest kink of any kind
    margin_energy: float = math.inf   # ... to the nearest discontinuity of the energy itself


def energy_and_gradient(grid: Grid, lig, genes, want_margin=True) -> EvalResult:
    genes = np.asarray(genes, dtype=np.float64)
    n = lig.n_atoms
    x = pose(lig, genes)
    # grid part
    e_atoms, F, s_atoms, Fabs = grid_energies(grid, x, lig.types, lig.charges, with_force_scale=True)
    e_inter = float(e_atoms.sum())
    scale = float(s_atoms.sum())
    margin = margin_e = math.inf
    if want_margin:
        ins, g = inside(grid, x)
        ins = np.atleast_1d(ins)
        margin_e = min(float(np.min(np.abs(g))), float(np.min(np.abs(g - (grid.n_xyz - 1)))))
        margin = margin_e
        if np.any(ins):
            frac = g[ins] - np.floor(g[ins])
            margin = min(margin, float(np.min(np.minimum(frac, 1.0 - frac))))
    # pair part
    e_intra = 0.0
    if lig.pairs.shape[0]:
        i, j = lig.pairs[:, 0], lig.pairs[:, 1]
        d = x[i] - x[j]
        r = np.sqrt(np.sum(d * d, axis=1))
        is_hb, c12, cn, qq, ds = pair_table(lig)
        e, dedr, s, _ = pair_energy(r, is_hb, c12, cn, qq, ds)
        e_intra = float(e.sum())
        scale += float(s.sum())
        f = np.where(dedr[:, None] != 0.0, dedr[:, None] * d / np.where(r > 0, r, 1.0)[:, None], 0.0)
        np.add.at(F, i, f)
        np.add.at(F, j, -f)
        np.add.at(Fabs, i, np.abs(f))
        np.add.at(Fabs, j, np.abs(f))
        if want_margin:
            margin_e = min(margin_e, float(np.min(np.abs(r - C.CUTOFF))), float(np.min(np.abs(r - C.CUTOFF_EL))))
            margin = min(margin, margin_e, float(np.min(np.abs(r - C.R_MIN))))

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
                      e_intra=e_intra, scale_energy=scale, scale_grad=sgrad, margin=margin,
                      margin_energy=margin_e)


def energy(grid: Grid, lig, genes) -> float:
    return energy_and_gradient(grid, lig, genes, want_margin=False).energy
