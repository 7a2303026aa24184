"""md_dock_noalloc: the dock whose workspace is the library's static device array, called through
the C ABI, against md_dock (the same kernels, so the same results bit for bit), on two calls in a
row -- the second with a smaller input, so it reuses the array the first one left behind -- and
its refusal of a dock that needs more workspace than the array holds."""
import numpy as np
import pytest

from workload import configs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2203_02096_amd as m
    m.lib()
    return m


def _same(a, b):
    for k in ("best_energy", "best_genes", "best_xyz", "run_index", "evals", "generations"):
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_equals_md_dock_twice(md):
    rec = configs.receptor("plain_fp32_small")
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    tp = configs.type_params()
    # first a larger dock, then a smaller ligand with fewer runs and a smaller population
    cases = [(synth.make_ligand(45, 9, 8101, tp), dict(n_runs=6, pop_size=60, max_generations=4, ls_rate=0.1,
                                                        ls_iters=40, seed=11)),
             (synth.make_ligand(14, 3, 8102, tp), dict(n_runs=3, pop_size=20, max_generations=3, ls_rate=0.2,
                                                        ls_iters=25, seed=12))]
    for lig, kw in cases:
        dlig = md.Ligand.from_synth(lig)
        P = md.dock_params(**configs.search_params("plain_fp32_small", **kw))
        want = md.md_dock(drec, dlig, P)
        got = md.md_dock_noalloc(drec, dlig, P)
        _same(got, want)
        assert np.all(np.diff(got["best_energy"]) >= 0)
        assert sorted(got["run_index"].tolist()) == list(range(kw["n_runs"]))


def test_noalloc_mixed_local_search_and_no_xyz(md):
    rec = configs.receptor("plain_fp32_small")
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    dlig = md.Ligand.from_synth(synth.make_ligand(70, 12, 8103, configs.type_params()))   # two atoms per lane
    P = md.dock_params(**configs.search_params("plain_fp32_small", n_runs=4, pop_size=30, max_generations=2,
                                               ls_rate=0.1, ls_iters=30, seed=13, ls_method=1))
    want = md.md_dock(drec, dlig, P, want_xyz=False)
    got = md.md_dock_noalloc(drec, dlig, P, want_xyz=False)
    _same(got, want)


def test_noalloc_rejects_oversized_dock(md):
    rec = configs.receptor("plain_fp32_small")
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    dlig = md.Ligand.from_synth(synth.make_ligand(40, 8, 8104, configs.type_params()))
    # 200 runs x 1000 individuals x 15 genes x 2 populations x 4 B = 24 MB > 8 MiB
    P = md.dock_params(**configs.search_params("plain_fp32_small", n_runs=200, pop_size=1000, max_generations=1,
                                               seed=14))
    with pytest.raises(md.MdockError) as ei:
        md.md_dock_noalloc(drec, dlig, P)
    assert ei.value.status == md.mdock.MD_ERANGE
    assert "scratch" in str(ei.value)
