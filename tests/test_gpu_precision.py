"""Grid maps stored in FP16 / BF16 (interpolation, accumulation and gradient stay FP32):
error against the FP64 oracle, split into the kernel's own error (oracle on the same rounded
maps, held to the FP32 tolerance) and the total error (oracle on the FP32 maps, bounded by
the rounding of the map values that each interpolation touches)."""
import sys

import numpy as np
import pytest

from parity_util import compare, oracle_eval_many, oracle_ligand
from oracle import scoring as S
from workload import configs, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def round_maps(maps, precision):
    """The stored values, as the library rounds them (round to nearest even)."""
    m = np.asarray(maps, np.float32)
    if precision == "fp16":
        return m.astype(np.float16).astype(np.float64)
    bits = m.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16 << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


UNIT_ROUNDOFF = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2203_02096_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
@pytest.mark.parametrize("lig_case", [(40, 8, 202), (70, 20, 601), (15, 3, 602)], ids=["40a", "70a", "15a"])
def test_low_precision_maps(md, precision, lig_case):
    na, nt, seed = lig_case
    rec = synth.make_receptor(64, 102)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, precision)
    lig = synth.make_ligand(na, nt, seed, configs.type_params())
    dlig = md.Ligand.from_synth(lig)
    n = 301
    genes = synth.random_genes(lig, rec, n, seed=seed, margin=2.0)
    e = torch.empty(n, device="cuda")
    d = torch.empty(n, lig.n_genes, device="cuda")
    md.md_eval(drec, dlig, torch.from_numpy(genes).cuda(), e, d)
    torch.cuda.synchronize()
    E, D = e.cpu().numpy(), d.cpu().numpy()
    ol = oracle_ligand(lig)
    # kernel-only error: the oracle on the rounded maps, to the FP32 tolerance
    rounded = S.make_grid(round_maps(rec.maps, precision), rec.origin, rec.spacing)
    ref_r = oracle_eval_many(rounded, ol, genes)
    stats = compare(ref_r, E, D)
    # total error: the oracle on the FP32 maps; bound = FP32 tolerance + rounding of every
    # map value touched (unit roundoff x the grid part's condition scale)
    exact = S.make_grid(rec.maps, rec.origin, rec.spacing)
    ref = oracle_eval_many(exact, ol, genes)
    u = UNIT_ROUNDOFF[precision]
    rel = []
    for p, r in enumerate(ref):
        if r.margin_energy < 5e-5:
            continue
        grid_scale = sum(S.grid_energies(exact, r.x, ol.types, ol.charges)[2])
        err = abs(float(E[p]) - r.energy)
        assert err <= 1e-4 * max(abs(r.energy), r.scale_energy) + u * grid_scale, (p, err)
        rel.append(err / max(abs(r.energy), r.scale_energy))
    _say(f"[{precision} maps] ligand {na} atoms: kernel-only {stats}; total energy error vs FP32 "
         f"maps: median {np.median(rel):.2e}, max {np.max(rel):.2e} (relative to the condition scale)")


def test_low_precision_dock_drift(md):
    """Best-energy drift versus the FP32 path.  At fixed poses (the FP32 search's best pose of
    every run) the FP16/BF16 energies stay within the rounding bound of the FP32 ones; the
    searches' own best energies (re-scored by the oracle on the FP32 maps) are reported."""
    rec = synth.make_receptor(64, 102)
    lig = configs.ligand("plain_fp32_production")
    dlig = md.Ligand.from_synth(lig)
    P = md.dock_params(**configs.search_params("plain_fp32_production", n_runs=8, max_generations=6,
                                               max_evals_per_run=10 ** 12, seed=21))
    grid = S.make_grid(rec.maps, rec.origin, rec.spacing)
    ol = oracle_ligand(lig)
    recs = {p: md.Receptor(rec.maps, rec.origin, rec.spacing, p) for p in ("fp32", "fp16", "bf16")}
    runs = {p: md.md_dock(recs[p], dlig, P) for p in recs}
    best32 = runs["fp32"]["best_genes"]
    g = torch.from_numpy(np.ascontiguousarray(best32)).cuda()
    e = {}
    for p, drec in recs.items():
        out = torch.empty(g.shape[0], device="cuda")
        md.md_eval(drec, dlig, g, out, None)
        torch.cuda.synchronize()
        e[p] = out.cpu().numpy()
    for p in ("fp16", "bf16"):
        for k in range(g.shape[0]):
            r = S.energy_and_gradient(grid, ol, best32[k].astype(np.float64))
            bound = UNIT_ROUNDOFF[p] * sum(S.grid_energies(grid, r.x, ol.types, ol.charges)[2]) \
                + 2e-4 * max(abs(r.energy), r.scale_energy)
            assert abs(float(e[p][k]) - float(e["fp32"][k])) <= bound, (p, k)
    rescored = {p: S.energy(grid, ol, runs[p]["best_genes"][0].astype(np.float64)) for p in recs}
    _say(f"[precision drift] at the FP32 best poses: max |E16 - E32| = "
         f"{np.abs(e['fp16'] - e['fp32']).max():.3e}, max |Ebf16 - E32| = {np.abs(e['bf16'] - e['fp32']).max():.3e} "
         f"kcal/mol; search outcomes re-scored on FP32 maps: {rescored}")
