"""GPU parity of the Solis-Wets local search (md_local_search_sw and the GA with
ls_method = Solis-Wets) against the FP64 oracle on the same seeded inputs and the same
counter-based normals.

Solis-Wets moves by steps that do not depend on the current point, so FP32 and FP64 searches
from one start stay together (their points differ by rounding only) for as long as they take
the same accept/reject decisions.  A decision compares two energies; each side's energy is
within the evaluation tolerance of the exact one, so the two sides can decide differently
only where the oracle's two energies are within twice that tolerance of each other (a near
tie), or where an evaluated point sits within KINK of a place where the energy jumps.  The
parity test therefore compares every evaluation element by element up to the first
disagreement and requires that disagreement to follow a near tie or a kink."""
import sys

import numpy as np
import pytest

from parity_util import E_TOL, check_sw_start, oracle_grid, oracle_ligand
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


_REC = {}


def _receptor(md, n, seed):
    if (n, seed) not in _REC:
        rec = synth.make_receptor(n, seed)
        _REC[(n, seed)] = (rec, md.Receptor(rec.maps, rec.origin, rec.spacing))
    return _REC[(n, seed)]


def _run_gpu(md, drec, dlig, genes, n_evals, seed):
    gin = torch.from_numpy(genes).cuda()
    gout = torch.empty_like(gin)
    eout = torch.empty(genes.shape[0], device="cuda")
    trace = torch.empty(genes.shape[0], n_evals, device="cuda")
    md.md_local_search_sw(drec, dlig, gin, gout, eout, n_evals, seed, trace)
    torch.cuda.synchronize()
    return gout.cpu().numpy(), eout.cpu().numpy(), trace.cpu().numpy()


# (name, grid, map seed, atoms, torsions, ligand seed, starts, evaluations)
SW_CASES = [
    ("small_20a_4t", 40, 101, 20, 4, 201, 13, 200),
    ("production_40a_8t", 64, 102, 40, 8, 202, 8, 300),
    ("max_128a_32t", 64, 102, 128, 32, 304, 4, 120),
    ("rigid_30a_0t", 40, 101, 30, 0, 307, 5, 120),
    ("tiny_1a", 40, 101, 1, 0, 308, 5, 150),
]


@pytest.mark.parametrize("case", SW_CASES, ids=[c[0] for c in SW_CASES])
def test_solis_wets_parity(md, case):
    name, gn, gseed, na, nt, lseed, n, n_evals = case
    rec, drec = _receptor(md, gn, gseed)
    lig = synth.make_ligand(na, nt, lseed, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    genes = synth.random_genes(lig, rec, n, seed=lseed + 1, margin=4.0)
    seed = 1000 + lseed
    G, E, T = _run_gpu(md, drec, dlig, genes, n_evals, seed)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    agree = []
    for k in range(n):
        d, cause = check_sw_start(grid, ol, genes[k], G[k], E[k], T[k], n_evals, seed, k)
        agree.append(d)
        _say(f"[sw parity] {name} start {k}: {d}/{n_evals} evaluations agree (first cause: {cause}); "
             f"E {T[k, 0]:.5g} -> {E[k]:.5g}")
    # the searches really are compared: most evaluations of most starts agree
    assert np.median(agree) >= min(n_evals, 60)


def test_solis_wets_budget_edges(md):
    """n_evals = 1 returns the start unchanged; n_evals = 2 tries x + xi only; no start is a
    no-op; the budget is rejected above 2^24."""
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand("plain_fp32_small")
    dlig = md.Ligand.from_synth(lig)
    genes = synth.random_genes(lig, rec, 6, seed=5, margin=4.0)
    G1, E1, T1 = _run_gpu(md, drec, dlig, genes, 1, 3)
    assert np.array_equal(G1, genes) and np.array_equal(E1, T1[:, 0])
    G2, E2, T2 = _run_gpu(md, drec, dlig, genes, 2, 3)
    assert np.array_equal(T2[:, 0], T1[:, 0])
    assert np.array_equal(E2, np.minimum(T2[:, 0], T2[:, 1]))
    for k in range(6):
        if T2[k, 1] >= T2[k, 0]:
            assert np.array_equal(G2[k], genes[k])
    empty = torch.empty(0, genes.shape[1], device="cuda")
    md.md_local_search_sw(drec, dlig, empty, empty, torch.empty(0, device="cuda"), 10, 1)
    x = torch.from_numpy(genes).cuda()
    with pytest.raises(md.MdockError):
        md.md_local_search_sw(drec, dlig, x, x, torch.empty(6, device="cuda"), (1 << 24) + 1, 1)


def test_solis_wets_deterministic_and_seeded(md):
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand("plain_fp32_small")
    dlig = md.Ligand.from_synth(lig)
    genes = synth.random_genes(lig, rec, 9, seed=8, margin=4.0)
    a = _run_gpu(md, drec, dlig, genes, 100, 21)
    b = _run_gpu(md, drec, dlig, genes, 100, 21)
    c = _run_gpu(md, drec, dlig, genes, 100, 22)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[2], c[2])


def _sw_params(md, name, **kw):
    return md.dock_params(**configs.search_params(name, ls_method="solis_wets", **kw))


def test_dock_solis_wets_matches_oracle(md):
    """Two GA generations with Solis-Wets on 20 % of the population: the same picks, the same
    normals, the same best individual as the oracle's GA."""
    from oracle import lga as OG
    from oracle import scoring as S
    name = "plain_fp32_small"
    rec, drec = _receptor(md, 40, 101)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    kw = dict(n_runs=2, pop_size=40, max_generations=2, ls_rate=0.2, ls_iters=20, seed=5)
    res = md.md_dock(drec, dlig, _sw_params(md, name, **kw))
    ref = OG.lga_dock(oracle_grid(rec), oracle_ligand(lig), OG.DockParams(**kw, ls_method="solis_wets"))
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    for k in range(2):
        _say(f"[dock sw 2 gens] gpu {res['best_energy'][k]:.6g} (run {res['run_index'][k]}) "
             f"ref {ref['best_energy'][k]:.6g} (run {ref['order'][k]})")
        scale = S.energy_and_gradient(grid, ol, ref["best_genes"][k]).scale_energy
        assert res["run_index"][k] == ref["order"][k]
        assert abs(res["best_energy"][k] - ref["best_energy"][k]) <= E_TOL * max(abs(ref["best_energy"][k]), scale)
        assert np.allclose(res["best_genes"][k], ref["best_genes"][k], atol=1e-4)
        assert res["evals"][k] == 40 + 2 * (39 + 8 * 20)


def test_dock_solis_wets_production_accounting(md):
    """The production workload with Solis-Wets: closed-form evaluation counts, deterministic,
    reported energies are the oracle's energies of the reported poses."""
    from oracle import scoring as S
    name = "plain_fp32_production"
    rec, drec = _receptor(md, 64, 102)
    lig = configs.ligand(name)
    dlig = md.Ligand.from_synth(lig)
    P = _sw_params(md, name, seed=7, n_runs=4)
    r1 = md.md_dock(drec, dlig, P)
    r2 = md.md_dock(drec, dlig, P)
    assert np.all(r1["evals"] == 150 + 56 * 45149)
    assert np.array_equal(r1["best_genes"], r2["best_genes"])
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    for k in range(4):
        ref = S.energy_and_gradient(grid, ol, r1["best_genes"][k].astype(np.float64))
        assert abs(ref.energy - r1["best_energy"][k]) <= E_TOL * max(abs(ref.energy), ref.scale_energy)
    ra = md.md_dock(drec, dlig, md.dock_params(**configs.search_params(name, seed=7, n_runs=4)))
    _say(f"[dock production] best energies Solis-Wets {r1['best_energy']}, ADADELTA {ra['best_energy']}")


def _mixed_jobs(md):
    """ADADELTA and Solis-Wets jobs of four sizes."""
    sizes = [(10, 3), (40, 8), (65, 14), (100, 32)]
    ligs = [synth.make_ligand(n, t, 600 + k, configs.type_params()) for k, (n, t) in enumerate(sizes)]
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    jobs = []
    for k, dl in enumerate(dligs):
        for method in ("adadelta", "solis_wets"):
            jobs.append((dl, md.dock_params(**configs.search_params(
                "batched_fp32", n_runs=2, pop_size=40, max_generations=3, ls_rate=0.2, ls_iters=40,
                seed=70 + k, ls_method=method))))
    return jobs


def test_batch_mixed_local_searches_equal_alone(md):
    """ADADELTA and Solis-Wets jobs of several sizes in one batch (separate launch classes)
    give bitwise the same answers as each job docked alone."""
    rec, drec = _receptor(md, 64, 102)
    jobs = _mixed_jobs(md)
    batch = md.md_dock_batch(drec, jobs)
    for k, (dl, p) in enumerate(jobs):
        alone = md.md_dock(drec, dl, p)
        for key in ("best_energy", "best_genes", "run_index", "evals", "generations"):
            assert np.array_equal(batch[k][key], alone[key]), (k, key)
    assert not np.array_equal(batch[0]["best_genes"], batch[1]["best_genes"])
