"""The file front end end to end on the GPU: a receptor read from nine AutoGrid map texts and the
ring ligand of tests/golden/ligand_ring.pdbqt with the type parameters of
tests/golden/atom_par_test.dat, through the library's readers, evaluated and docked; the oracle
gets the same maps as arrays and the ligand as the hand reading of the fixture
(tests/golden/ligand_ring.json), so no oracle input passes through the library."""
import numpy as np
import pytest

from oracle import ligand as OL
from oracle import scoring as S
from workload import configs, synth

from parity_util import clean_genes, compare
from test_formats import _golden, autogrid_text, expected_ligand

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2203_02096_amd as m
    m.lib()
    return m


def _inputs(md):
    rec = synth.make_receptor(41, 5151)
    center = np.asarray(rec.origin) + 0.5 * (np.asarray(rec.shape_xyz) - 1) * rec.spacing
    texts = [autogrid_text(rec.maps[m], rec.spacing, center) for m in range(rec.maps.shape[0])]
    drec = md.receptor_from_autogrid(texts)
    exp = expected_ligand()
    tp_lib = md.md_atom_par_parse(_golden("atom_par_test.dat"), exp["type_names"])
    dlig = md.ligand_from_pdbqt(_golden("ligand_ring.pdbqt"), exp["type_names"], tp_lib)
    tp = np.asarray(exp["type_params_from_atom_par_test"], np.float32)
    bonds = np.asarray(exp["bonds"], np.int32)
    tors = np.asarray([exp["bonds"].index(b) for b in exp["torsion_bonds"]], np.int32)
    lig = synth.Ligand(np.asarray(exp["xyz"], np.float32), np.asarray(exp["types"], np.int32),
                       np.asarray(exp["charges"], np.float32), bonds, tors, 0, tp)
    ol = OL.prepare(lig.xyz, lig.types, lig.charges, lig.bonds, lig.torsions, tp, root=0)
    grid = S.make_grid(rec.maps, rec.origin, rec.spacing)
    return rec, drec, dlig, lig, ol, grid


def test_ring_ligand_from_files_matches_oracle(md):
    import torch
    rec, drec, dlig, lig, ol, grid = _inputs(md)
    assert dlig.n_atoms == 12 and dlig.n_genes == 10 and dlig.n_pairs == len(ol.pairs)
    genes, _ = clean_genes(lig, rec, 48, seed=61, olig=ol, grid=grid)
    g = torch.from_numpy(genes).cuda()
    e = torch.empty(len(genes), device="cuda")
    d = torch.empty(len(genes), lig.n_genes, device="cuda")
    md.md_eval(drec, dlig, g, e, d)
    torch.cuda.synchronize()
    ref = [S.energy_and_gradient(grid, ol, x.astype(np.float64)) for x in genes]
    stats = compare(ref, e.cpu().numpy(), d.cpu().numpy())
    assert stats["checked_energy"] >= 40 and stats["checked"] >= 40


def test_ring_ligand_from_files_docks(md):
    rec, drec, dlig, lig, ol, grid = _inputs(md)
    P = md.dock_params(**configs.search_params("plain_fp32_small", n_runs=4, pop_size=40, max_generations=5,
                                               ls_rate=0.1, ls_iters=60, seed=21))
    res = md.md_dock(drec, dlig, P)
    assert np.all(np.diff(res["best_energy"]) >= 0)
    for k in range(4):
        r = S.energy_and_gradient(grid, ol, res["best_genes"][k].astype(np.float64))
        assert abs(res["best_energy"][k] - r.energy) <= 1e-4 * max(abs(r.energy), r.scale_energy)
