"""Launch plans and the autotuner: every plan (waves per block, waves per pose, LDS budget -- from
all pair rows read from global memory to all staged in up to 160 KiB of LDS -- and lane-group
size) gives
energies and gradients within the parity tolerance of the FP64 oracle, with the energy-only and
gradient paths bitwise equal; the autotuner picks one of them, records it for the size class,
and a dock with a tuned plan is reproducible."""
import sys

import numpy as np
import pytest

from parity_util import compare, oracle_eval_many, oracle_grid, oracle_ligand
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
    m.md_tune_table_clear()
    yield m
    m.md_tune_table_clear()


@pytest.fixture(scope="module")
def receptor(md):
    rec = synth.make_receptor(64, 102)
    return rec, md.Receptor(rec.maps, rec.origin, rec.spacing)


PLANS = [dict(lds_budget=0, group_div=3, waves_per_block=4),
         dict(lds_budget=160 * 1024, group_div=3, waves_per_block=8),
         dict(lds_budget=32 * 1024, group_div=2, waves_per_block=1),
         dict(lds_budget=96 * 1024, group_div=4, waves_per_block=2),
         dict(lds_budget=65536, group_div=8, waves_per_block=8),
         # the widest blocks: 16 waves (12 for more than 64 atoms), one block per compute unit
         dict(lds_budget=160 * 1024, group_div=3, waves_per_block=16),
         dict(lds_budget=160 * 1024, group_div=2, waves_per_block=12),
         # waves sharing a pose (the block holds one pose)
         dict(lds_budget=65536, group_div=3, waves_per_block=2, waves_per_pose=2),
         dict(lds_budget=160 * 1024, group_div=3, waves_per_block=4, waves_per_pose=4),
         dict(lds_budget=0, group_div=2, waves_per_block=4, waves_per_pose=4)]


@pytest.mark.parametrize("na,nt", [(22, 4), (66, 14), (110, 30)])
def test_every_plan_matches_oracle(md, receptor, na, nt):
    rec, drec = receptor
    lig = synth.make_ligand(na, nt, 1200 + na, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    n = 67                                   # two partial blocks for every waves-per-block choice
    genes = synth.random_genes(lig, rec, n, seed=na, margin=2.0)
    ref = oracle_eval_many(oracle_grid(rec), oracle_ligand(lig), genes)
    g_dev = torch.from_numpy(genes).cuda()
    for plan in PLANS:
        info = md.md_ligand_set_plan(dlig, **plan)
        _say(f"[plans] {na} atoms: {info}")
        e = torch.empty(n, device="cuda")
        d = torch.empty(n, lig.n_genes, device="cuda")
        e2 = torch.empty(n, device="cuda")
        md.md_eval(drec, dlig, g_dev, e, d)
        md.md_eval(drec, dlig, g_dev, e2, None)
        torch.cuda.synchronize()
        E, D, E2 = e.cpu().numpy(), d.cpu().numpy(), e2.cpu().numpy()
        assert np.array_equal(E, E2), plan
        stats = compare(ref, E, D)
        assert stats["checked_energy"] >= 0.9 * n, plan


def test_local_search_consistent_across_plans(md, receptor):
    """The local search under two very different plans: each result's energy is the energy of
    its returned genotype (md_eval, same plan), and both sets are close to each other."""
    rec, drec = receptor
    lig = synth.make_ligand(48, 9, 1301, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    n = 96
    genes = torch.from_numpy(synth.random_genes(lig, rec, n, seed=5, margin=3.0)).cuda()
    outs = []
    for plan in (PLANS[0], PLANS[1], PLANS[6]):
        md.md_ligand_set_plan(dlig, **plan)
        go = torch.empty_like(genes)
        eo = torch.empty(n, device="cuda")
        md.md_local_search(drec, dlig, genes, go, eo, 40)
        ee = torch.empty(n, device="cuda")
        md.md_eval(drec, dlig, go, ee, None)
        torch.cuda.synchronize()
        assert np.array_equal(eo.cpu().numpy(), ee.cpu().numpy()), plan
        outs.append(eo.cpu().numpy())
    # the two searches follow the same iteration up to summation order: most end close together
    for other in outs[1:]:
        rel = np.abs(outs[0] - other) / np.maximum(1.0, np.abs(other))
        assert np.median(rel) < 1e-2


def test_autotune_and_table(md, receptor):
    rec, drec = receptor
    md.md_tune_table_clear()
    lig = synth.make_ligand(40, 8, 1401, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    info = md.md_ligand_autotune(drec, dlig)
    _say(f"[autotune] 40 atoms: {info}")
    assert not info["from_table"] and info["candidates"] >= 2
    assert 0 < info["us_per_eval"] <= info["default_us_per_eval"] * 1.0000001
    assert md.md_tune_table_size() == 1
    plan = md.md_ligand_get_plan(dlig)
    assert plan == info["plan"]
    # same class: creation keeps the default plan whatever the table holds; a second autotune
    # applies the table's plan untimed
    twin = md.Ligand.from_synth(synth.make_ligand(40, 8, 1402, configs.type_params()))
    fresh = md.Ligand.from_synth(synth.make_ligand(40, 8, 1402, configs.type_params()))
    assert md.md_ligand_get_plan(twin) == md.md_ligand_get_plan(fresh)
    assert md.md_ligand_get_plan(twin)["waves_per_block"] == 4 and md.md_ligand_get_plan(twin)["lds_budget"] == 65536
    again = md.md_ligand_autotune(drec, twin)
    assert again["from_table"]
    assert md.md_ligand_get_plan(twin)["waves_per_block"] == plan["waves_per_block"]
    assert md.md_ligand_get_plan(twin)["lds_budget"] == plan["lds_budget"]
    # parity after tuning
    genes = synth.random_genes(lig, rec, 65, seed=9, margin=2.0)
    e = torch.empty(65, device="cuda")
    d = torch.empty(65, lig.n_genes, device="cuda")
    md.md_eval(drec, dlig, torch.from_numpy(genes).cuda(), e, d)
    torch.cuda.synchronize()
    compare(oracle_eval_many(oracle_grid(rec), oracle_ligand(lig), genes), e.cpu().numpy(), d.cpu().numpy())
    # a dock with the tuned plan is reproducible
    P = md.dock_params(**configs.search_params("serving_fp16", n_runs=3, pop_size=40, max_generations=3,
                                               ls_rate=0.2, ls_iters=20, seed=3))
    a, b = md.md_dock(drec, dlig, P), md.md_dock(drec, dlig, P)
    for k in ("best_energy", "best_genes", "evals"):
        assert np.array_equal(a[k], b[k]), k
    md.md_tune_table_clear()
    assert md.md_tune_table_size() == 0


def test_batch_autotune(md, receptor):
    """The batch tuner times every policy on the batch, applies one, and afterwards a batch's
    results still equal each ligand docked alone; best energies re-scored by the oracle agree."""
    from oracle import scoring as S
    rec, drec = receptor
    sizes = [(14, 2), (36, 7), (70, 15), (52, 9), (95, 24), (25, 4)]
    ligs = [synth.make_ligand(n, t, 1500 + k, configs.type_params()) for k, (n, t) in enumerate(sizes)]
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    Ps = [md.dock_params(**configs.search_params("serving_fp16", n_runs=3, pop_size=40, max_generations=4,
                                                 ls_rate=0.2, ls_iters=20, seed=70 + k)) for k in range(len(ligs))]
    info = md.md_batch_autotune(drec, list(zip(dligs, Ps)), generations=4)
    _say(f"[batch autotune] {info}")
    assert info["policy"] in md.mdock.BATCH_POLICIES
    assert all(v > 0 for v in info["ms_per_generation"].values())
    batch = md.md_dock_batch(drec, list(zip(dligs, Ps)))
    grid = oracle_grid(rec)
    for k, (dl, P) in enumerate(zip(dligs, Ps)):
        alone = md.md_dock(drec, dl, P)
        for key in ("best_energy", "best_genes", "evals"):
            assert np.array_equal(batch[k][key], alone[key]), (k, key)
        r = S.energy_and_gradient(grid, oracle_ligand(ligs[k]), batch[k]["best_genes"][0].astype(np.float64))
        assert abs(float(batch[k]["best_energy"][0]) - r.energy) <= 1e-4 * max(abs(r.energy), r.scale_energy)
    md.md_tune_table_clear()


def test_creation_independent_of_tuning_history(md, receptor):
    """Two creations of one ligand, one before and one after a tuning call that records a plan
    for its size class, get the same plan and dock to bitwise the same result."""
    rec, drec = receptor
    md.md_tune_table_clear()
    lig = synth.make_ligand(52, 9, 1403, configs.type_params())
    P = md.dock_params(**configs.search_params("serving_fp16", n_runs=2, pop_size=30, max_generations=2,
                                               ls_rate=0.2, ls_iters=15, seed=8))
    before = md.Ligand.from_synth(lig)
    res_before = md.md_dock(drec, before, P)
    md.md_ligand_autotune(drec, md.Ligand.from_synth(synth.make_ligand(52, 9, 1404, configs.type_params())),
                          force=True)
    assert md.md_tune_table_size() == 1
    after = md.Ligand.from_synth(lig)
    assert md.md_ligand_get_plan(after) == md.md_ligand_get_plan(before)
    res_after = md.md_dock(drec, after, P)
    for k in ("best_energy", "best_genes", "best_xyz", "evals"):
        assert np.array_equal(res_before[k], res_after[k]), k
    md.md_tune_table_clear()
