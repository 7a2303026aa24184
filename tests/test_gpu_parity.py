"""GPU parity: libmdock's HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs."""
import math
import sys

import numpy as np
import pytest

from parity_util import (assert_xyz_is_pose, clean_genes, compare, oracle_eval_many, oracle_grid, oracle_ligand,
                         tolerance_over_grid_terms)
from workload import configs, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


_REC_CACHE = {}


def _receptor(md, grid_n, seed, precision="fp32"):
    key = (grid_n, seed, precision)
    if key not in _REC_CACHE:
        rec = synth.make_receptor(grid_n, seed)
        _REC_CACHE[key] = (rec, md.Receptor(rec.maps, rec.origin, rec.spacing, precision))
    return _REC_CACHE[key]


# (name, grid, map seed, atoms, torsions, ligand seed, poses)
EVAL_CASES = [
    ("small_20a_4t", 40, 101, 20, 4, 201, 401),
    ("production_40a_8t", 64, 102, 40, 8, 202, 203),
    ("wide_100a_32t", 64, 102, 100, 32, 303, 61),
    ("max_128a_32t", 64, 102, 128, 32, 304, 29),
    ("edge_64a_12t", 64, 102, 64, 12, 305, 41),
    ("edge_65a_12t", 64, 102, 65, 12, 306, 41),
    ("rigid_30a_0t", 40, 101, 30, 0, 307, 101),
    ("rigid_100a_0t", 64, 102, 100, 0, 311, 41),
    ("rigid_128a_0t", 64, 102, 128, 0, 312, 29),
    ("tiny_1a", 40, 101, 1, 0, 308, 67),
    ("tiny_2a", 40, 101, 2, 0, 309, 67),
    ("tiny_4a_1t", 40, 101, 4, 1, 310, 67),
]


def _eval_both(md, drec, dlig, genes):
    """md_eval with and without the gradient; the energies must agree bitwise."""
    n = genes.shape[0]
    g_dev = torch.from_numpy(genes).cuda()
    e_dev = torch.empty(n, device="cuda")
    d_dev = torch.empty(n, genes.shape[1], device="cuda")
    md.md_eval(drec, dlig, g_dev, e_dev, d_dev)
    e_only = torch.empty(n, device="cuda")
    md.md_eval(drec, dlig, g_dev, e_only, None)
    torch.cuda.synchronize()
    E, D, E2 = e_dev.cpu().numpy(), d_dev.cpu().numpy(), e_only.cpu().numpy()
    assert np.array_equal(E, E2), "energy-only and energy+gradient paths must agree bitwise"
    return E, D


@pytest.mark.parametrize("case", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_eval_parity(md, case):
    """Clean poses (every atom inside the grid, torsions near the clash-free reference, the
    tolerance at most 1 % of the in-grid atom terms): every energy and gradient within the
    tolerance rule, so an error of the grid term as a whole cannot pass."""
    name, gn, ms, na, nt, ls, npose = case
    _say(f"[eval parity clean] {name}: grid {gn}^3 atoms {na} torsions {nt} poses {npose}")
    rec, drec = _receptor(md, gn, ms)
    lig = synth.make_ligand(na, nt, ls, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    genes, tries = clean_genes(lig, rec, npose, seed=ls, olig=ol, grid=grid)
    E, D = _eval_both(md, drec, dlig, genes)
    ref = oracle_eval_many(grid, ol, genes)
    stats = compare(ref, E, D)
    power = [tolerance_over_grid_terms(grid, ol, r) for r in ref]
    _say(f"[eval parity clean] {name}: {stats}; {npose} clean of {tries} draws; "
         f"tolerance / sum|grid terms| median {np.median(power):.2e} max {np.max(power):.2e}")
    assert stats["checked_energy"] >= 0.9 * npose and stats["checked"] >= 0.75 * npose


@pytest.mark.parametrize("case", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_eval_parity_wild(md, case):
    """Edge cases: random poses anywhere in the box shrunk by 2 A -- atoms outside the grid (the
    out-of-grid penalty and its restoring gradient) and folded torsions (clashing pairs at the
    0.5 A clamp).  Same tolerance rule; here the clash and penalty terms dominate the scale."""
    name, gn, ms, na, nt, ls, npose = case
    _say(f"[eval parity wild] {name}: grid {gn}^3 atoms {na} torsions {nt} poses {npose}")
    rec, drec = _receptor(md, gn, ms)
    lig = synth.make_ligand(na, nt, ls, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    genes = synth.random_genes(lig, rec, npose, seed=ls, margin=2.0)
    E, D = _eval_both(md, drec, dlig, genes)
    ref = oracle_eval_many(oracle_grid(rec), oracle_ligand(lig), genes)
    stats = compare(ref, E, D)
    _say(f"[eval parity wild] {name}: {stats}")
    assert stats["checked_energy"] >= 0.9 * npose and stats["checked"] >= 0.75 * npose


def test_eval_zero_and_ragged(md):
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand("plain_fp32_small")
    dlig = md.Ligand.from_synth(lig)
    z = torch.empty(0, lig.n_genes, device="cuda")
    md.md_eval(drec, dlig, z, torch.empty(0, device="cuda"), None)
    genes = synth.random_genes(lig, rec, 7, seed=3)
    full = torch.empty(7, device="cuda")
    md.md_eval(drec, dlig, torch.from_numpy(genes).cuda(), full, None)
    for n in (1, 2, 3, 5):
        part = torch.empty(n, device="cuda")
        md.md_eval(drec, dlig, torch.from_numpy(genes[:n]).cuda(), part, None)
        torch.cuda.synchronize()
        assert np.array_equal(part.cpu().numpy(), full.cpu().numpy()[:n])


def test_pose_parity(md):
    from oracle import pose as OP
    rec = synth.make_receptor(40, 101)
    for na, nt, seed in [(20, 4, 201), (100, 32, 303), (128, 32, 304)]:
        lig = synth.make_ligand(na, nt, seed, configs.type_params())
        dlig = md.Ligand.from_synth(lig)
        genes = synth.random_genes(lig, rec, 33, seed=seed)
        xyz = torch.empty(33, na, 3, device="cuda")
        md.md_pose(dlig, torch.from_numpy(genes).cuda(), xyz)
        torch.cuda.synchronize()
        ol = oracle_ligand(lig)
        ref = np.stack([OP.pose(ol, g.astype(np.float64)) for g in genes])
        err = np.abs(xyz.cpu().numpy() - ref).max()
        _say(f"[pose parity] {na} atoms: max |dx| = {err:.2e} A")
        assert err < 2e-4


def test_local_search_parity(md):
    """ADADELTA from identical starts: the first steps agree to the evaluation tolerance, and
    the returned best energy agrees within the trajectory tolerance."""
    from oracle import adadelta as OA
    from oracle import scoring as S
    name = "plain_fp32_small"
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    n, iters = 6, 300
    genes = synth.random_genes(lig, rec, n, seed=77, margin=4.0)
    gin = torch.from_numpy(genes).cuda()
    gout = torch.empty_like(gin)
    eout = torch.empty(n, device="cuda")
    trace = torch.empty(n, iters, device="cuda")
    md.md_local_search(drec, dlig, gin, gout, eout, iters, 0.8, 1e-2, trace)
    torch.cuda.synchronize()
    G, Eb, Tr = gout.cpu().numpy(), eout.cpu().numpy(), trace.cpu().numpy()
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    for p in range(n):
        bx, be, traj = OA.local_search(grid, ol, genes[p].astype(np.float64), iters, 0.8, 1e-2, trace=True)
        te = np.array([e for e, _ in traj])
        scale0 = S.energy_and_gradient(grid, ol, genes[p].astype(np.float64)).scale_energy
        diverge = next((s for s in range(iters) if abs(Tr[p, s] - te[s]) > 1e-4 * max(abs(te[s]), scale0)), iters)
        _say(f"[ls parity] start {p}: E0 gpu {Tr[p,0]:.6g} ref {te[0]:.6g}; best gpu {Eb[p]:.6g} "
             f"ref {be:.6g}; first step off by >1e-4: {diverge}")
        assert abs(Tr[p, 0] - te[0]) <= 1e-4 * max(abs(te[0]), scale0)
        assert diverge >= 5
        # returned best is the minimum of the GPU's own trace, and its genes re-evaluate to it
        assert Eb[p] == Tr[p].min()
        re = S.energy_and_gradient(grid, ol, G[p].astype(np.float64))
        assert abs(re.energy - Eb[p]) <= 1e-4 * max(abs(re.energy), re.scale_energy)


def _dock_params(md, name, **over):
    p = configs.search_params(name, **over)
    return md.dock_params(**p)


def test_dock_initial_population(md):
    """No generation: the result is the best individual of the initial population, drawn from
    the same counter-based random numbers as the oracle."""
    from oracle import lga as OG
    from oracle import scoring as S
    name = "plain_fp32_small"
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    P = _dock_params(md, name, n_runs=3, pop_size=40, max_generations=0, seed=11)
    res = md.md_dock(drec, dlig, P)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    op = OG.DockParams(n_runs=3, pop_size=40, max_generations=0, seed=11)
    for k in range(3):
        r = int(res["run_index"][k])
        pop = [OG.initial_individual(grid, ol, op, r, i) for i in range(40)]
        E = [S.energy(grid, ol, x) for x in pop]
        b = OG.argbest(E)
        ref = S.energy_and_gradient(grid, ol, pop[b])
        assert abs(res["best_energy"][k] - E[b]) <= 1e-4 * max(abs(E[b]), ref.scale_energy)
        assert np.allclose(res["best_genes"][k], pop[b], atol=2e-5)
        assert res["evals"][k] == 40 and res["generations"][k] == 0
    assert np.all(np.diff(res["best_energy"]) >= 0)


def test_dock_one_generation_matches_oracle(md):
    """One GA generation without local search: selection, crossover and mutation consume the
    same random numbers as the oracle, so the best individual agrees."""
    from oracle import lga as OG
    name = "plain_fp32_small"
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    kw = dict(n_runs=2, pop_size=40, max_generations=2, ls_rate=0.0, seed=5)
    res = md.md_dock(drec, dlig, _dock_params(md, name, **kw))
    op = OG.DockParams(**{**kw, "ls_iters": 300})
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    ref = OG.lga_dock(grid, ol, op)
    from oracle import scoring as S
    for k in range(2):
        _say(f"[dock 2 gens] gpu {res['best_energy'][k]:.6g} (run {res['run_index'][k]}) "
             f"ref {ref['best_energy'][k]:.6g} (run {ref['order'][k]})")
        assert res["run_index"][k] == ref["order"][k]
        scale = S.energy_and_gradient(grid, ol, ref["best_genes"][k]).scale_energy
        assert abs(res["best_energy"][k] - ref["best_energy"][k]) <= 1e-4 * max(abs(ref["best_energy"][k]), scale)
        assert np.allclose(res["best_genes"][k], ref["best_genes"][k], atol=1e-4)
        assert res["evals"][k] == 40 + 2 * 39


def test_dock_eval_accounting_and_determinism(md):
    """The full small workload: per-run evaluation counts follow the closed form, and a
    second call with the same seed gives bitwise the same answer."""
    name = "plain_fp32_small"
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    P = _dock_params(md, name, seed=3)
    assert md.md_dock_planned_generations(P) == 10
    r1 = md.md_dock(drec, dlig, P)
    r2 = md.md_dock(drec, dlig, P)
    assert r1["evals"][0] == 150 + 10 * (149 + 9 * 300) == 28640
    assert r1["generations"][0] == 10
    assert np.array_equal(r1["best_genes"], r2["best_genes"])
    assert np.array_equal(r1["best_energy"], r2["best_energy"])
    # the reported energy is the energy of the reported pose
    from oracle import scoring as S
    ref = S.energy_and_gradient(oracle_grid(rec), oracle_ligand(lig), r1["best_genes"][0].astype(np.float64))
    assert abs(ref.energy - r1["best_energy"][0]) <= 1e-4 * max(abs(ref.energy), ref.scale_energy)
    _say(f"[dock small] best {r1['best_energy'][0]:.5g} kcal/mol")


def test_dock_production_sampled(md):
    """Full production workload (64^3 grid, 40 atoms / 8 torsions, 20 runs x 150, 2.5M evals per
    run, local search on every individual): counts follow the closed form, and every run's
    reported best energy equals the oracle's energy of the reported pose."""
    from oracle import scoring as S
    name = "plain_fp32_production"
    rec, drec = _receptor(md, 64, 102)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    P = _dock_params(md, name, seed=7)
    res = md.md_dock(drec, dlig, P)
    assert np.all(res["evals"] == 150 + 56 * 45149)
    assert np.all(np.diff(res["best_energy"]) >= 0)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    for k in range(P.n_runs):
        ref = S.energy_and_gradient(grid, ol, res["best_genes"][k].astype(np.float64))
        assert abs(ref.energy - res["best_energy"][k]) <= 1e-4 * max(abs(ref.energy), ref.scale_energy)
    _say(f"[dock production] best energies {res['best_energy'][:5]}")


BATCH_SIZES = [(10, 3), (30, 8), (64, 12), (65, 14), (100, 32)]


def test_dock_batch_equals_alone(md):
    """Ligands of different sizes docked in one batch give bitwise the same answer as each
    docked alone (their random numbers and arithmetic do not depend on the batch)."""
    rec, drec = _receptor(md, 64, 102)
    ligs = [synth.make_ligand(n, t, 400 + k, configs.type_params()) for k, (n, t) in enumerate(BATCH_SIZES)]
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    params = [md.dock_params(**configs.search_params("batched_fp32", n_runs=3, pop_size=40,
                                                     max_generations=3, ls_rate=0.2, ls_iters=40,
                                                     seed=50 + k)) for k in range(len(ligs))]
    batch = md.md_dock_batch(drec, list(zip(dligs, params)))
    for k in range(len(ligs)):
        assert_xyz_is_pose(md, dligs[k], batch[k])
        alone = md.md_dock(drec, dligs[k], params[k])
        assert_xyz_is_pose(md, dligs[k], alone)
        _say(f"[batch] ligand {BATCH_SIZES[k]}: best {batch[k]['best_energy'][0]:.5g} alone {alone['best_energy'][0]:.5g}")
        for key in ("best_energy", "best_genes", "best_xyz", "run_index", "evals", "generations"):
            assert np.array_equal(batch[k][key], alone[key]), (k, key)
        assert np.all(batch[k]["evals"] == 40 + 3 * (39 + 8 * 40))


def test_dock_batch_energies_match_oracle(md):
    """Every job's reported best energy is the oracle's energy of its reported pose, and its
    reported coordinates are the oracle's pose of its reported genes."""
    from oracle import pose as OP
    from oracle import scoring as S
    rec, drec = _receptor(md, 64, 102)
    ligs = [synth.make_ligand(n, t, 500 + k, configs.type_params()) for k, (n, t) in enumerate(BATCH_SIZES)]
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    params = [md.dock_params(**configs.search_params("batched_fp32", n_runs=2, pop_size=30,
                                                     max_generations=2, ls_rate=0.1, ls_iters=30,
                                                     seed=9)) for _ in ligs]
    res = md.md_dock_batch(drec, list(zip(dligs, params)))
    grid = oracle_grid(rec)
    for lig, r in zip(ligs, res):
        ol = oracle_ligand(lig)
        for k in range(2):
            g = r["best_genes"][k].astype(np.float64)
            ref = S.energy_and_gradient(grid, ol, g)
            if ref.margin_energy >= 5e-5:
                assert abs(ref.energy - r["best_energy"][k]) <= 1e-4 * max(abs(ref.energy), ref.scale_energy)
            assert np.abs(r["best_xyz"][k] - OP.pose(ol, g)).max() < 2e-4


def test_dock_batch_rejects_bad_job(md):
    rec, drec = _receptor(md, 40, 101)
    lig = md.Ligand.from_synth(configs.ligand("plain_fp32_small"))
    good = md.dock_params(**configs.search_params("plain_fp32_small", max_generations=1))
    bad = md.dock_params(**configs.search_params("plain_fp32_small", pop_size=1))
    with pytest.raises(md.MdockError, match="job 1"):
        md.md_dock_batch(drec, [(lig, good), (lig, bad)])


def test_batched_workload_full_shape_sampled(md):
    """The batched workload at its full shape (256 ligands of 10-100 atoms against the 64^3 maps,
    10 runs x 150 each, 6 % local search x 300) for 3 generations through md_dock_batch, as the
    batched bench launches it: every job's evaluation count follows the closed form, and for 16
    jobs spread over the batch every run's reported best energy is the oracle's energy of the
    reported pose."""
    from oracle import scoring as S
    name = "batched_fp32"
    rec, drec = _receptor(md, 64, 102)
    ligs = configs.batched_ligands(name)
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    P = md.dock_params(**configs.search_params(name, seed=11, max_generations=3))
    res = md.md_dock_batch(drec, [(d, P) for d in dligs], want_xyz=False)
    per_gen = (150 - 1) + 9 * 300
    for r in res:
        assert np.all(r["evals"] == 150 + 3 * per_gen)
        assert np.all(np.diff(r["best_energy"]) >= 0)
    grid = oracle_grid(rec)
    checked = 0
    for k in np.linspace(0, len(ligs) - 1, 16).astype(int):
        ol = oracle_ligand(ligs[k])
        for run in range(P.n_runs):
            ref = S.energy_and_gradient(grid, ol, res[k]["best_genes"][run].astype(np.float64))
            if ref.margin_energy >= 5e-5:
                assert abs(ref.energy - res[k]["best_energy"][run]) <= 1e-4 * max(abs(ref.energy), ref.scale_energy)
                checked += 1
    _say(f"[batched full shape] {checked} sampled run bests re-scored by the oracle")
    assert checked >= 0.9 * 16 * P.n_runs
