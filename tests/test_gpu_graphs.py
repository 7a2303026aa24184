"""HIP-graph generations: md_dock / md_dock_batch capture one LGA generation and replay it.  Every
result must equal the kernel-by-kernel launch order bitwise, after any number of replays, with
eager device work and synchronisations between calls.  (The server's branch launch against
kernel-by-kernel ticks is in test_gpu_zz_server.py.)"""
import sys

import numpy as np
import pytest

from workload import configs, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("best_energy", "best_genes", "best_xyz", "run_index", "evals", "generations")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2203_02096_amd as m
    m.lib()
    yield m
    m.md_set_graphs(True)


@pytest.fixture(scope="module")
def receptor(md):
    rec = synth.make_receptor(64, 102)
    return rec, md.Receptor(rec.maps, rec.origin, rec.spacing)


def _dock(md, drec, lig, P, graphs):
    md.md_set_graphs(graphs)
    try:
        return md.md_dock(drec, lig, P)
    finally:
        md.md_set_graphs(True)


@pytest.mark.parametrize("gens", [2, 3, 7])
def test_dock_graph_replays_equal_eager(md, receptor, gens):
    rec, drec = receptor
    lig = md.Ligand.from_synth(synth.make_ligand(30, 6, 901, configs.type_params()))
    P = md.dock_params(**configs.search_params("serving_fp16", n_runs=4, pop_size=40, max_generations=gens,
                                               ls_rate=0.25, ls_iters=25, seed=31 + gens))
    _say(f"[graphs] md_dock 30 atoms, {gens} generations: eager then graph")
    eager = _dock(md, drec, lig, P, False)
    x = torch.randn(1 << 20, device="cuda")       # unrelated eager work between the calls
    (x * 2).sum().item()
    graph = _dock(md, drec, lig, P, True)
    torch.cuda.synchronize()
    again = _dock(md, drec, lig, P, True)
    for k in KEYS:
        assert np.array_equal(eager[k], graph[k]), k
        assert np.array_equal(graph[k], again[k]), k
    assert int(eager["generations"][0]) == gens


def test_dock_batch_graph_equals_eager(md, receptor):
    """Mixed sizes across the size classes (one and two atoms per lane, several LDS classes)."""
    rec, drec = receptor
    sizes = [(12, 2), (40, 8), (70, 16), (25, 4), (100, 20), (55, 10)]
    ligs = [md.Ligand.from_synth(synth.make_ligand(n, t, 910 + k, configs.type_params()))
            for k, (n, t) in enumerate(sizes)]
    Ps = [md.dock_params(**configs.search_params("serving_fp16", n_runs=3, pop_size=30, max_generations=4,
                                                 ls_rate=0.2, ls_iters=20, seed=40 + k)) for k in range(len(ligs))]
    _say("[graphs] md_dock_batch of 6 ligands, eager then graph")
    md.md_set_graphs(False)
    eager = md.md_dock_batch(drec, list(zip(ligs, Ps)))
    md.md_set_graphs(True)
    graph = md.md_dock_batch(drec, list(zip(ligs, Ps)))
    for k in range(len(ligs)):
        for key in KEYS:
            assert np.array_equal(eager[k][key], graph[k][key]), (k, key)


def test_profiled_batch_equals_graph(md, receptor):
    """A profiled batch (each GA phase's size-class launches concurrent over the branch streams,
    each phase timed) gives bitwise the results of the captured graph; small size classes join a
    larger class's launches either way (the plans below give several LDS classes of few waves)."""
    rec, drec = receptor
    sizes = [(12, 2), (40, 8), (70, 16), (25, 4), (100, 20), (55, 10), (18, 3)]
    ligs = [md.Ligand.from_synth(synth.make_ligand(n, t, 930 + k, configs.type_params()))
            for k, (n, t) in enumerate(sizes)]
    md.md_ligand_set_plan(ligs[0], lds_budget=160 * 1024, waves_per_block=4)
    md.md_ligand_set_plan(ligs[3], lds_budget=32 * 1024, waves_per_block=4)
    md.md_ligand_set_plan(ligs[6], lds_budget=160 * 1024, waves_per_block=16)
    Ps = [md.dock_params(**configs.search_params("serving_fp16", n_runs=3, pop_size=30, max_generations=5,
                                                 ls_rate=0.2, ls_iters=20, seed=60 + k)) for k in range(len(ligs))]
    _say("[graphs] md_dock_batch of 7 ligands, graph then profiled")
    md.md_set_graphs(True)
    graph = md.md_dock_batch(drec, list(zip(ligs, Ps)))
    md.md_profile_reset()
    md.md_profile_enable(True)
    try:
        prof = md.md_dock_batch(drec, list(zip(ligs, Ps)))
    finally:
        md.md_profile_enable(False)
    ms, n = md.md_profile_read("local_search")
    assert n == 5 and ms > 0          # one timed local-search phase per generation
    for k in range(len(ligs)):
        for key in KEYS:
            assert np.array_equal(graph[k][key], prof[k][key]), (k, key)
