"""Waves sharing a pose (plans with waves_per_pose 2 or 4): the local searches, the evaluation
entry point and whole docks against the FP64 oracle, and against the one-wave-per-pose plan.
Sharing changes only the order of the force and energy sums, so every comparison uses the
same tolerance rule as the one-wave path."""
import sys

import numpy as np
import pytest

from parity_util import E_TOL, check_sw_start, compare, oracle_eval_many, oracle_grid, oracle_ligand
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


@pytest.fixture(scope="module")
def receptor(md):
    rec = synth.make_receptor(64, 102)
    return rec, md.Receptor(rec.maps, rec.origin, rec.spacing)


def _share(md, dlig, wpp, lds_budget=65536):
    return md.md_ligand_set_plan(dlig, lds_budget=lds_budget, group_div=3, waves_per_block=wpp, waves_per_pose=wpp)


# (atoms, torsions, ligand seed): one and two atoms per lane, the largest ligand, no pairs
SIZES = [(22, 4, 2101), (66, 14, 2102), (128, 32, 2103), (1, 0, 2104), (3, 0, 2105)]


@pytest.mark.parametrize("na,nt,seed", SIZES, ids=[f"{a}a_{t}t" for a, t, _ in SIZES])
@pytest.mark.parametrize("wpp", [2, 4])
def test_eval_parity(md, receptor, na, nt, seed, wpp):
    rec, drec = receptor
    lig = synth.make_ligand(na, nt, seed, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    info = _share(md, dlig, wpp, lds_budget=32 * 1024 if na > 100 else 65536)
    assert info["waves_per_pose"] == wpp and info["waves_per_block"] == wpp
    n = 37
    genes = synth.random_genes(lig, rec, n, seed=seed, margin=2.0)
    g_dev = torch.from_numpy(genes).cuda()
    e, d, e2 = torch.empty(n, device="cuda"), torch.empty(n, lig.n_genes, device="cuda"), torch.empty(n, device="cuda")
    md.md_eval(drec, dlig, g_dev, e, d)
    md.md_eval(drec, dlig, g_dev, e2, None)
    torch.cuda.synchronize()
    E, D, E2 = e.cpu().numpy(), d.cpu().numpy(), e2.cpu().numpy()
    assert np.array_equal(E, E2)
    stats = compare(oracle_eval_many(oracle_grid(rec), oracle_ligand(lig), genes), E, D)
    _say(f"[share eval] {na} atoms, {wpp} waves per pose: {info['staged_rows']}/{info['total_rows']} rows "
         f"staged, worst energy {stats.get('worst_energy', 0):.2e}")
    assert stats["checked_energy"] >= 0.9 * n


@pytest.mark.parametrize("wpp", [2, 4])
def test_adadelta_parity(md, receptor, wpp):
    """ADADELTA with a shared pose from identical starts: the first steps agree with the oracle's
    to the evaluation tolerance; the returned genotype re-evaluates to the returned energy.
    From heavily clashing random starts (energies up to 1e9) a gene whose gradient is small
    against its condition scale takes an FP32 step that differs from the FP64 one, so a
    trajectory may leave the oracle's after two steps; this happens alike with one wave per pose
    (measured on these starts), so every start must agree for two steps and the median start
    for five."""
    from oracle import adadelta as OA
    from oracle import scoring as S
    rec, drec = receptor
    grid = oracle_grid(rec)
    for na, nt, seed in SIZES[:3]:
        lig = synth.make_ligand(na, nt, seed, configs.type_params())
        dlig = md.Ligand.from_synth(lig)
        _share(md, dlig, wpp)
        ol = oracle_ligand(lig)
        n, iters = 5, 80
        genes = synth.random_genes(lig, rec, n, seed=seed + 7, margin=4.0)
        gin = torch.from_numpy(genes).cuda()
        gout, eout = torch.empty_like(gin), torch.empty(n, device="cuda")
        trace = torch.empty(n, iters, device="cuda")
        md.md_local_search(drec, dlig, gin, gout, eout, iters, 0.8, 1e-2, trace)
        torch.cuda.synchronize()
        G, Eb, Tr = gout.cpu().numpy(), eout.cpu().numpy(), trace.cpu().numpy()
        agreed = []
        for p in range(n):
            _, _, traj = OA.local_search(grid, ol, genes[p].astype(np.float64), iters, 0.8, 1e-2, trace=True)
            te = np.array([e for e, _ in traj])
            sc = S.energy_and_gradient(grid, ol, genes[p].astype(np.float64)).scale_energy
            agree = next((s for s in range(iters) if abs(Tr[p, s] - te[s]) > E_TOL * max(abs(te[s]), sc)), iters)
            _say(f"[share adadelta] {na} atoms, {wpp} waves: start {p} agrees for {agree} steps")
            assert abs(Tr[p, 0] - te[0]) <= E_TOL * max(abs(te[0]), sc)
            assert agree >= 2
            agreed.append(agree)
            assert Eb[p] == Tr[p].min()
            re = S.energy_and_gradient(grid, ol, G[p].astype(np.float64))
            assert abs(re.energy - Eb[p]) <= E_TOL * max(abs(re.energy), re.scale_energy)
        assert np.median(agreed) >= 5


def test_solis_wets_parity(md, receptor):
    """Solis-Wets with four waves per pose: every evaluation agrees with the oracle's up to a near
    tie or kink."""
    rec, drec = receptor
    grid = oracle_grid(rec)
    for na, nt, seed in SIZES[:3]:
        lig = synth.make_ligand(na, nt, seed, configs.type_params())
        dlig = md.Ligand.from_synth(lig)
        _share(md, dlig, 4)
        ol = oracle_ligand(lig)
        n, n_evals, sseed = 4, 120, 31
        genes = synth.random_genes(lig, rec, n, seed=seed + 9, margin=4.0)
        gin = torch.from_numpy(genes).cuda()
        gout, eout = torch.empty_like(gin), torch.empty(n, device="cuda")
        trace = torch.empty(n, n_evals, device="cuda")
        md.md_local_search_sw(drec, dlig, gin, gout, eout, n_evals, sseed, trace)
        torch.cuda.synchronize()
        G, E, T = gout.cpu().numpy(), eout.cpu().numpy(), trace.cpu().numpy()
        agree = []
        for k in range(n):
            d, cause = check_sw_start(grid, ol, genes[k], G[k], E[k], T[k], n_evals, sseed, k)
            agree.append(d)
            _say(f"[share sw] {na} atoms: start {k}: {d}/{n_evals} agree ({cause})")
        assert np.median(agree) >= 60


def test_docks_with_shared_poses(md, receptor):
    """Docks whose local searches share poses: closed-form counts, reported energies re-evaluate,
    reproducible; a batch mixing shared and unshared plans equals each ligand docked alone; the
    dock stays within the tolerance of the unshared plan's first generation."""
    from oracle import scoring as S
    rec, drec = receptor
    grid = oracle_grid(rec)
    ligs = [synth.make_ligand(na, nt, seed + 50, configs.type_params()) for na, nt, seed in SIZES[:3]]
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    for dl, wpp in zip(dligs, (2, 4, 4)):
        _share(md, dl, wpp)
    jobs, of = [], []
    for k, dl in enumerate(dligs):
        for method in ("adadelta", "solis_wets"):
            jobs.append((dl, md.dock_params(**configs.search_params(
                "paper_inputs", n_runs=3, pop_size=40, max_generations=3, ls_rate=0.2, ls_iters=30,
                seed=90 + k, ls_method=method))))
            of.append(oracle_ligand(ligs[k]))
    extra = md.Ligand.from_synth(ligs[1])            # same ligand, one wave per pose
    jobs.append((extra, jobs[2][1]))
    of.append(oracle_ligand(ligs[1]))
    batch = md.md_dock_batch(drec, jobs)
    for k, (dl, P) in enumerate(jobs):
        alone = md.md_dock(drec, dl, P)
        again = md.md_dock(drec, dl, P)
        for key in ("best_energy", "best_genes", "run_index", "evals", "generations"):
            assert np.array_equal(batch[k][key], alone[key]), (k, key)
            assert np.array_equal(again[key], alone[key]), (k, key)
        assert np.all(alone["evals"] == 40 + 3 * (39 + 8 * 30))
        for r in range(3):
            ref = S.energy_and_gradient(grid, of[k], alone["best_genes"][r].astype(np.float64))
            if ref.margin_energy >= 5e-5:
                assert abs(ref.energy - alone["best_energy"][r]) <= E_TOL * max(abs(ref.energy), ref.scale_energy)
    _say(f"[share dock] 66 atoms ADADELTA best: 2 waves per pose {batch[2]['best_energy'][0]:.4f}, "
         f"1 wave {batch[-1]['best_energy'][0]:.4f}")
