"""ADADELTA parity at every step, despite chaos.

Two FP32 and FP64 searches from one start drift apart after a few steps (the energy surface
amplifies rounding), so comparing the library's whole trajectory with the oracle's says nothing
past the first steps.  Instead the oracle shadows the library's own trajectory: the library
records every iterate x_s and the gradient g_s its update used (md_local_search_traced), and at
every one of the 300 steps
  * the oracle's FP64 energy and gradient at x_s must match the library's (E_s, g_s) under the
    evaluation tolerance rule, and
  * the oracle's ADADELTA update (memetic local search; Zeiler 2012, Algorithm 1; accumulators
    fed the library's own gradients) from x_s must land on the library's x_{s+1}: quaternion
    renormalised, torsions wrapped, within FP32 rounding of the step;
and the returned best genotype and energy must be the first minimum of the recorded energies."""
import math
import sys

import numpy as np
import pytest

from parity_util import clean_genes, compare, oracle_eval_many, oracle_grid, oracle_ligand
from workload import configs, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RHO, EPS, ITERS = 0.8, 1e-2, 300


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2203_02096_amd as m
    m.lib()
    return m


def _shadow_updates(X, Gr, n_tors):
    """Worst step error over the trace of one search: the oracle's ADADELTA update from each
    recorded iterate with the recorded gradient, against the next recorded iterate.  Returns
    (worst error / allowed, steps checked)."""
    from oracle import adadelta as OA
    x = X[0].astype(np.float64)
    eg2 = np.zeros_like(x)
    edx2 = np.zeros_like(x)
    worst = 0.0
    for s in range(X.shape[0] - 1):
        xs = X[s].astype(np.float64)
        g = Gr[s].astype(np.float64)
        nx, eg2, edx2 = OA.adadelta_step(xs, g, eg2, edx2, RHO, EPS)
        step = nx - xs
        nx = OA.project_genes(nx, n_tors)
        got = X[s + 1].astype(np.float64)
        d = got - nx
        d[7:] = (d[7:] + math.pi) % (2 * math.pi) - math.pi      # torsions: on the circle
        # FP32 rounding of the genes (a few ulp of |x|) plus a relative error of the step from
        # the FP32 accumulators and the hardware square roots
        allowed = 4e-7 * (np.abs(nx) + 1.0) + 1e-4 * np.abs(step)
        worst = max(worst, float(np.max(np.abs(d) / allowed)))
    return worst, X.shape[0] - 1


CASES = [("small_20a_4t", 40, 101, 20, 4, 201, 6, 1), ("production_40a_8t", 64, 102, 40, 8, 202, 4, 1),
         ("two_slots_100a_24t", 64, 102, 100, 24, 303, 3, 1), ("shared_pose_40a_8t_w2", 64, 102, 40, 8, 202, 3, 2),
         ("shared_pose_66a_14t_w4", 64, 102, 66, 14, 305, 2, 4)]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adadelta_every_step_shadowed(md, case):
    name, gn, ms, na, nt, ls, n, wpp = case
    _say(f"[adadelta shadow] {name}: {n} searches x {ITERS} steps, waves per pose {wpp}")
    rec = synth.make_receptor(gn, ms)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    lig = synth.make_ligand(na, nt, ls, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    if wpp > 1:
        md.md_ligand_set_plan(dlig, waves_per_pose=wpp)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    starts, _ = clean_genes(lig, rec, n, seed=ls + 17, olig=ol, grid=grid)
    G = lig.n_genes
    gin = torch.from_numpy(starts).cuda()
    gout, eout = torch.empty_like(gin), torch.empty(n, device="cuda")
    tr = torch.empty(n, ITERS, device="cuda")
    tx = torch.empty(n, ITERS, G, device="cuda")
    tg = torch.empty(n, ITERS, G, device="cuda")
    md.md_local_search_traced(drec, dlig, gin, gout, eout, ITERS, RHO, EPS, tr, tx, tg)
    torch.cuda.synchronize()
    E, X, Gr = tr.cpu().numpy(), tx.cpu().numpy(), tg.cpu().numpy()
    gbest, ebest = gout.cpu().numpy(), eout.cpu().numpy()
    for p in range(n):
        assert np.array_equal(X[p, 0], starts[p])
        # every iterate's evaluation
        ref = oracle_eval_many(grid, ol, X[p])
        stats = compare(ref, E[p], Gr[p])
        assert stats["checked_energy"] >= 0.9 * ITERS and stats["checked"] >= 0.75 * ITERS, stats
        # every update
        worst, steps = _shadow_updates(X[p], Gr[p], lig.n_torsions)
        # the result: the first lowest recorded energy and its iterate
        k = int(np.argmin(E[p]))
        assert ebest[p] == E[p, k] and np.array_equal(gbest[p], X[p, k])
        _say(f"[adadelta shadow] {name} start {p}: E {E[p, 0]:.4g} -> best {ebest[p]:.4g} at step {k}; "
             f"eval {stats['checked_energy']}/{ITERS} checked, worst E {stats['worst_energy']:.2e}, "
             f"worst g {stats['worst_grad']:.2e}; update worst {worst:.3f} of allowed over {steps} steps")
        assert worst <= 1.0
        assert np.allclose(np.linalg.norm(X[p, 1:, 3:7], axis=1), 1.0, atol=1e-6)
        assert np.all(X[p, 1:, 7:] > -math.pi - 1e-6) and np.all(X[p, 1:, 7:] <= math.pi + 1e-6)


def test_traced_search_equals_untraced(md):
    """Recording the trace changes nothing: the same results as md_local_search, bit for bit."""
    rec = synth.make_receptor(64, 102)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    lig = synth.make_ligand(40, 8, 202, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    starts = synth.random_genes(lig, rec, 9, seed=5, margin=4.0)
    gin = torch.from_numpy(starts).cuda()
    outs = []
    for traced in (False, True):
        go, eo = torch.empty_like(gin), torch.empty(9, device="cuda")
        tr = torch.empty(9, 50, device="cuda")
        if traced:
            tx = torch.empty(9, 50, lig.n_genes, device="cuda")
            md.md_local_search_traced(drec, dlig, gin, go, eo, 50, RHO, EPS, tr, tx, None)
        else:
            md.md_local_search(drec, dlig, gin, go, eo, 50, RHO, EPS, tr)
        torch.cuda.synchronize()
        outs.append((go.cpu().numpy(), eo.cpu().numpy(), tr.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
