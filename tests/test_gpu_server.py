"""Continuous-batching server: requests that arrive while others run are admitted as slots and
memory free up, and each result is the same as docking the request alone."""
import sys
import time

import numpy as np
import pytest

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


SIZES = [(12, 2), (25, 5), (40, 8), (64, 12), (70, 16), (33, 6), (90, 24), (18, 3)]


def _params(md, k, **over):
    kw = dict(n_runs=3, pop_size=30, max_generations=3, ls_rate=0.2, ls_iters=30, seed=100 + k)
    kw.update(over)
    return md.dock_params(**configs.search_params("serving_fp16", **kw))


def test_server_results_equal_alone(md, receptor):
    rec, drec = receptor
    ligs = [md.Ligand.from_synth(synth.make_ligand(n, t, 700 + k, configs.type_params()))
            for k, (n, t) in enumerate(SIZES)]
    srv = md.Server(drec, hbm_budget_bytes=256 << 20, max_slots=4)
    tickets = []
    for k, lig in enumerate(ligs):
        tickets.append(srv.submit(lig, _params(md, k)))
        time.sleep(0.002 * k)          # staggered arrivals while earlier requests run
    results = [srv.wait(t, timeout_s=120) for t in tickets]
    st = srv.stats()
    srv.close()
    _say(f"[server] stats {st}")
    assert st["completed"] == len(ligs)
    for k, lig in enumerate(ligs):
        alone = md.md_dock(drec, lig, _params(md, k))
        for key in ("best_energy", "best_genes", "best_xyz", "run_index", "evals", "generations"):
            assert np.array_equal(results[k][key], alone[key]), (k, key)


def test_server_admission_by_memory(md, receptor):
    """A pool that holds two requests' buffers (but not three): never more than two requests
    resident at once, and every request still completes."""
    rec, drec = receptor
    lig = md.Ligand.from_synth(synth.make_ligand(30, 6, 801, configs.type_params()))
    kw = dict(n_runs=16, pop_size=512, max_generations=2, ls_iters=20)
    G, N, rows, runs = lig.n_genes, lig.n_atoms, 16 * 512, 16
    n_ls = int(np.ceil(0.2 * 512 - 1e-4))
    # a request's buffers: two populations, two energy arrays, counters, picks, results
    need = 2 * rows * G * 4 + 3 * rows * 4 + runs * 8 + runs * n_ls * 4 + 2 * runs * 4 \
        + runs * G * 4 + runs * N * 12
    budget = int(2.5 * need)          # alignment adds well under 1 % here
    assert budget >= (1 << 20)
    srv = md.Server(drec, hbm_budget_bytes=budget, max_slots=16)
    tickets = [srv.submit(lig, _params(md, k, **kw)) for k in range(6)]
    for t in tickets:
        srv.wait(t, timeout_s=120, want_xyz=False)
    spans = [srv.times(t)[1:] for t in tickets]
    srv.close()
    events = sorted([(a, 1) for a, _ in spans] + [(b, -1) for _, b in spans], key=lambda e: (e[0], e[1]))
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    _say(f"[server admission] budget {budget} B, request ~{need} B, peak resident {peak}")
    assert 1 <= peak <= 2


def test_server_cancel_and_errors(md, receptor):
    rec, drec = receptor
    lig = md.Ligand.from_synth(synth.make_ligand(40, 8, 802, configs.type_params()))
    srv = md.Server(drec, hbm_budget_bytes=64 << 20, max_slots=1)
    long_t = srv.submit(lig, _params(md, 0, max_generations=400))
    queued_t = srv.submit(lig, _params(md, 1))
    srv.cancel(queued_t)
    with pytest.raises(md.MdockError, match="cancel"):
        srv.wait(queued_t, timeout_s=30)
    srv.cancel(long_t)
    with pytest.raises(md.MdockError, match="cancel"):
        srv.wait(long_t, timeout_s=60)
    ok = srv.submit(lig, _params(md, 2))
    r = srv.wait(ok, timeout_s=60)
    assert r["generations"][0] == 3
    srv.close()
    small = md.Server(drec, hbm_budget_bytes=1 << 20, max_slots=1)
    with pytest.raises(md.MdockError, match="budget"):
        small.submit(lig, _params(md, 3, n_runs=50, pop_size=1000))
    small.close()
