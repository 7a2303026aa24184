"""Shared helpers of the GPU parity tests: oracle evaluation of many poses and the
acceptance rule for energies and gradients.

Tolerance rule (energies 1e-4, gradients 1e-3, relative): the reference value of a pose is a
sum of many terms of both signs (a clash term can reach 1e9 kcal/mol while the total is a few
kcal/mol), so "relative" is taken against the larger of |reference| and the sum of the
absolute values of the terms that make it up (the oracle's condition scale):
    |E_gpu - E_ref| <= 1e-4 * max(|E_ref|, S_E)
    |g_gpu - g_ref| <= 1e-3 * max(|g_ref|, S_k)     per gene k.
FP32 evaluation of such a sum carries an error of a few ulp of S, so the rule bounds what the
arithmetic can deliver; the plain relative error against |E_ref| is reported beside it.
The energy is piecewise smooth.  A pose whose FP32 coordinates could fall on the other side of
a kink than the FP64 ones is compared only where the compared quantity is continuous there:
energies are skipped within KINK of a grid box face or a hard cutoff (the energy jumps),
gradients also within KINK of a trilinear cell face or the 0.5 A clamp (the gradient jumps).
KINK = 5e-5 (grid units for faces, Angstrom for distances) is several times the FP32 error of a
posed coordinate in these boxes (|x| <= 20 A: 8 ulp ~ 1.5e-5 A ~ 4e-5 grid units).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ligand as OL
from oracle import scoring as S

E_TOL = 1e-4
G_TOL = 1e-3
KINK = 5e-5


def oracle_grid(rec):
    return S.make_grid(rec.maps, rec.origin, rec.spacing)


def oracle_ligand(lig):
    return OL.from_synth(lig)


def oracle_eval_many(grid, olig, genes):
    return [S.energy_and_gradient(grid, olig, np.asarray(g, np.float64)) for g in genes]


def compare(ref, e_gpu, g_gpu=None):
    """Returns a dict of error statistics; raises AssertionError on a violation."""
    n = len(ref)
    checked = checked_e = 0
    worst_e = worst_g = 0.0
    plain_e = []
    fails = []
    for p in range(n):
        r = ref[p]
        scale_e = max(abs(r.energy), r.scale_energy)
        err_e = abs(float(e_gpu[p]) - r.energy) / scale_e
        if r.margin_energy >= KINK:
            worst_e = max(worst_e, err_e)
            if err_e > E_TOL:
                fails.append(("energy", p, float(e_gpu[p]), r.energy, err_e))
            plain_e.append(abs(float(e_gpu[p]) - r.energy) / max(abs(r.energy), 1e-30))
            checked_e += 1
        if r.margin >= KINK:
            if g_gpu is not None:
                scale_g = np.maximum(np.abs(r.grad), r.scale_grad)
                err_g = np.abs(np.asarray(g_gpu[p], np.float64) - r.grad) / np.maximum(scale_g, 1e-30)
                worst_g = max(worst_g, float(err_g.max()))
                if np.any(err_g > G_TOL):
                    k = int(np.argmax(err_g))
                    fails.append(("grad", p, k, float(g_gpu[p][k]), r.grad[k], float(err_g[k])))
            checked += 1
    stats = dict(n=n, checked=checked, checked_energy=checked_e, worst_energy=worst_e, worst_grad=worst_g,
                 median_plain_rel_energy=float(np.median(plain_e)) if plain_e else 0.0)
    assert not fails, (fails[:5], stats)
    return stats


def check_sw_start(grid, ol, start, g_out, e_out, tr_gpu, n_evals, seed, k):
    """Solis-Wets from one start (standalone key (seed, 0, 0, k)): compares the library's energy
    trace tr_gpu with the oracle's element by element; the first disagreement must follow a near
    tie (two compared oracle energies within the sum of their tolerances) or a kink.  Checks the
    returned genotype and energy.  Returns (evaluations that agree, cause of the first
    disagreement)."""
    from oracle import scoring as S
    from oracle import solis_wets as OSW
    pts = []
    _, _, tr = OSW.local_search_sw(grid, ol, start.astype(np.float64), n_evals, seed, 0, 0, k,
                                   trace=True, points=pts)
    evs = [S.energy_and_gradient(grid, ol, x) for x in pts]
    tol = [E_TOL * max(abs(r.energy), r.scale_energy) for r in evs]
    d = next((i for i in range(n_evals) if evs[i].margin_energy >= KINK and abs(tr_gpu[i] - tr[i]) > tol[i]),
             n_evals)
    if d < n_evals:
        cause = None
        run_min = tr[0]
        for i in range(1, d + 1):
            if evs[i].margin_energy < KINK:
                cause = f"kink at evaluation {i}"
                break
            if i < d and abs(tr[i] - run_min) <= tol[i] + tol[int(np.argmin(tr[:i]))]:
                cause = f"near tie at evaluation {i} (|dE| {abs(tr[i] - run_min):.2e})"
                break
            run_min = min(run_min, tr[i])
        assert cause is not None, (k, d, tr_gpu[d], tr[d])
    else:
        cause = "none"
    # the result is the lowest energy the GPU evaluated, at a valid genotype that re-evaluates to it
    assert e_out == tr_gpu.min()
    re = S.energy_and_gradient(grid, ol, g_out.astype(np.float64))
    if re.margin_energy >= KINK:
        assert abs(re.energy - e_out) <= E_TOL * max(abs(re.energy), re.scale_energy)
    assert abs(np.linalg.norm(g_out[3:7]) - 1) < 1e-5
    assert np.all(g_out[7:] > -math.pi - 1e-6) and np.all(g_out[7:] <= math.pi + 1e-6)
    return d, cause


# The serving worker thread crashed the host process (SIGSEGV in that thread, no GPU fault) twice
# while it captured generation graphs; the cause is not known.  Capture in the worker is switched
# off, and the test that was running at the second crash stays off the GPU until a cause is shown.
SERVER_OFF_REASON = ("md_server's worker thread crashed the host process (SIGSEGV in that thread) while "
                     "this test ran, with graph capture in the worker; cause not known, held back")


def assert_xyz_is_pose(md, dlig, res):
    """A dock result's best_xyz must be the library's own pose (md_pose) of its best_genes, bit
    for bit: both come from one posing routine, and a mismatch means the coordinates were taken
    from other genes than the ones returned."""
    import torch
    genes = torch.from_numpy(np.ascontiguousarray(res["best_genes"], np.float32)).cuda()
    xyz = torch.empty(genes.shape[0], dlig.n_atoms, 3, device="cuda")
    md.md_pose(dlig, genes, xyz)
    torch.cuda.synchronize()
    want = xyz.cpu().numpy()
    bad = np.argwhere(np.any(res["best_xyz"] != want, axis=(1, 2))).ravel()
    assert bad.size == 0, ("best_xyz is not the pose of best_genes in runs", bad.tolist())


# Clean poses.  Random genotypes (workload.synth.random_genes) mostly put atoms outside the grid
# or fold torsions into clashes, and a clash or out-of-grid term can be 1e2-1e5 times the sum of
# all in-grid atom terms, so the tolerance above (relative to the sum of |terms|) would then not
# see an error of the whole grid term.  A clean pose has (a) every atom at least one grid spacing
# inside every face of the box, (b) torsion angles within CLEAN_TWIST of the reference
# conformation (which the ligand generator builds with every non-bonded distance >= 2 A) and
# (c) an energy tolerance at most CLEAN_POWER times the sum of |in-grid atom terms|, so that an
# error of that size in the grid term fails the comparison.  (A floor on pair distances such as
# 0.8 R_ij cannot be met: the 1-4 pairs of these ligands sit at 0.53-0.62 R_ij already in the
# reference conformation.)
CLEAN_TWIST = 0.3
CLEAN_POWER = 1e-2


def clean_genes(lig, rec, n, seed, olig=None, grid=None, max_tries=None):
    """n clean genotypes [n][7+T] float32 for ligand `lig` (workload.synth.Ligand) in receptor
    `rec`; orientation uniform, translation uniform over the placements that keep the ligand's
    box inside the grid, torsions uniform within CLEAN_TWIST.  Returns (genes, tries)."""
    from oracle import pose as OP
    olig = olig or oracle_ligand(lig)
    grid = grid or oracle_grid(rec)
    rng = np.random.default_rng([seed, 0xC1EA])
    lo = np.asarray(rec.origin, np.float64)
    hi = lo + (np.asarray(rec.shape_xyz, np.float64) - 1) * rec.spacing
    T = lig.n_torsions
    out, tries = [], 0
    max_tries = max_tries or 50 * n
    while len(out) < n:
        tries += 1
        assert tries <= max_tries, f"clean poses: {len(out)} of {n} after {tries} draws"
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        g = np.concatenate([[0.0, 0.0, 0.0], q, rng.uniform(-CLEAN_TWIST, CLEAN_TWIST, T)])
        x = OP.pose(olig, g)
        tlo = lo + rec.spacing - x.min(axis=0)
        thi = hi - rec.spacing - x.max(axis=0)
        if np.any(tlo >= thi):
            continue
        g[0:3] = rng.uniform(tlo, thi)
        g = g.astype(np.float32).astype(np.float64)   # the GPU gets these float32 genes
        r = S.energy_and_gradient(grid, olig, g)
        e_atoms, _, _ = S.grid_energies(grid, r.x, olig.types, olig.charges)
        if E_TOL * max(abs(r.energy), r.scale_energy) > CLEAN_POWER * float(np.sum(np.abs(e_atoms))):
            continue
        out.append(g)
    return np.asarray(out, np.float32).reshape(n, lig.n_genes), tries


def tolerance_over_grid_terms(grid, olig, r):
    """The energy tolerance of an oracle result r over the sum of |in-grid atom terms| of its
    pose: how large a grid-term error, relative to the grid term, the comparison would miss."""
    e_atoms, _, _ = S.grid_energies(grid, r.x, olig.types, olig.charges)
    return E_TOL * max(abs(r.energy), r.scale_energy) / max(float(np.sum(np.abs(e_atoms))), 1e-300)
