"""The file front end on the host: AutoGrid map files, PDBQT ligands and atom_par records
(md_autogrid_map_parse, md_pdbqt_parse, md_atom_par_parse), checked against hand readings of the
fixtures in tests/golden/ and against maps written out and read back; and ligands with rings,
which such files bring (rotatable bonds outside rings), in the library and in the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import ligand as OL
from workload import synth

md = pytest.importorskip("paper_2203_02096_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lib_available():
    try:
        md.lib()
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not _lib_available(), reason="libmdock.so not built")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return f.read()


def expected_ligand():
    return json.loads(_golden("ligand_ring.json"))


def autogrid_text(values_zyx, spacing, center, header=True):
    """An AutoGrid map file's text for values [nz][ny][nx] (x fastest), written here for the
    tests (the test writes the format, the library reads it)."""
    nz, ny, nx = values_zyx.shape
    lines = []
    if header:
        lines += ["GRID_PARAMETER_FILE test.gpf", "GRID_DATA_FILE test.maps.fld", "MACROMOLECULE test.pdbqt",
                  f"SPACING {spacing}", f"NELEMENTS {nx - 1} {ny - 1} {nz - 1}",
                  f"CENTER {center[0]:.6f} {center[1]:.6f} {center[2]:.6f}"]
    lines += ["%.9g" % v for v in np.asarray(values_zyx, np.float32).reshape(-1)]
    return "\n".join(lines) + "\n"


# ------------------------------------------------------------------ PDBQT
def test_pdbqt_matches_hand_reading():
    exp = expected_ligand()
    p = md.md_pdbqt_parse(_golden("ligand_ring.pdbqt"), exp["type_names"])
    assert np.array_equal(p["xyz"], np.asarray(exp["xyz"], np.float32))
    assert np.array_equal(p["charges"], np.asarray(exp["charges"], np.float32))
    assert p["types"].tolist() == exp["types"]
    assert p["serial"].tolist() == list(range(1, 13))
    assert p["root"] == exp["root"]
    got = sorted(tuple(sorted(b)) for b in p["bonds"].tolist())
    assert got == sorted(tuple(b) for b in exp["bonds"])
    tors = [tuple(sorted(p["bonds"][t].tolist())) for t in p["torsions"]]
    assert tors == [tuple(b) for b in exp["torsion_bonds"]]


def test_pdbqt_errors():
    names = expected_ligand()["type_names"]
    text = _golden("ligand_ring.pdbqt")
    bad = {
        "unknown type": text.replace(" OA\n", " Xx\n"),
        "unmatched branch": text.replace("ENDBRANCH   1   7\n", ""),
        "no root": text.replace("ROOT\n", "").replace("ENDROOT\n", ""),
        "short record": text.replace("ATOM      5 C5   LIG A   1      -0.695  -1.204   0.000", "ATOM      5 C5"),
        "branch atom missing": text.replace("BRANCH   7  10", "BRANCH   7  40").replace("ENDBRANCH   7  10",
                                                                                       "ENDBRANCH   7  40"),
        "unknown record": text.replace("TORSDOF 3", "CONECT 1 2"),
        "serial twice": text.replace("ATOM     12 H12", "ATOM     11 H12"),
    }
    for what, t in bad.items():
        with pytest.raises(md.MdockError) as ei:
            md.md_pdbqt_parse(t, names)
        assert ei.value.status == md.mdock.MD_EINVAL, what
    with pytest.raises(md.MdockError) as ei:
        md.md_pdbqt_parse(text, names, max_atoms=11)
    assert ei.value.status == md.mdock.MD_ERANGE


# ------------------------------------------------------------------ atom_par
def test_atom_par_matches_hand_reading():
    exp = expected_ligand()
    tp = md.md_atom_par_parse(_golden("atom_par_test.dat"), exp["type_names"])
    assert np.array_equal(tp, np.asarray(exp["type_params_from_atom_par_test"], np.float32))


def test_atom_par_missing_type():
    with pytest.raises(md.MdockError) as ei:
        md.md_atom_par_parse(_golden("atom_par_test.dat"), ["A", "C", "HD", "N", "NA", "OA", "Br"])
    assert "Br" in str(ei.value)


# ------------------------------------------------------------------ AutoGrid maps
def test_autogrid_map_round_trip():
    rec = synth.make_receptor(17, 4242)          # 16 intervals per axis, centred on the origin
    center = np.asarray(rec.origin) + 0.5 * (np.asarray(rec.shape_xyz) - 1) * rec.spacing
    for m in range(rec.maps.shape[0]):
        desc, vals = md.md_autogrid_map_parse(autogrid_text(rec.maps[m], rec.spacing, center))
        assert desc["shape"] == rec.shape_xyz
        assert desc["spacing"] == np.float32(rec.spacing)
        assert np.allclose(desc["origin"], rec.origin, atol=1e-6)
        assert np.array_equal(vals, rec.maps[m])


def test_autogrid_map_geometry_by_hand():
    # NELEMENTS 2 4 6 -> 3 x 5 x 7 nodes; origin = CENTER - SPACING * n / 2 per axis
    vals = np.arange(3 * 5 * 7, dtype=np.float32).reshape(7, 5, 3) * 0.25 - 3.0
    text = "SPACING 0.5\nNELEMENTS 2 4 6\nCENTER 1.0 -2.0 3.5\n" + autogrid_text(vals, 0.5, (0, 0, 0), header=False)
    desc, got = md.md_autogrid_map_parse(text)
    assert desc["shape"] == (3, 5, 7)
    assert desc["origin"] == pytest.approx((0.5, -3.0, 2.0))
    assert np.array_equal(got, vals)
    assert got[0, 0, 1] == vals.reshape(-1)[1]      # x fastest


def test_autogrid_map_errors():
    vals = np.zeros((3, 3, 3), np.float32)
    good = autogrid_text(vals, 0.375, (0, 0, 0))
    for t in (good.replace("NELEMENTS 2 2 2", "NELEMENTS 3 2 2"),      # odd interval count
              good.replace("SPACING 0.375\n", ""),                     # no spacing
              good + "1.0\n",                                          # one value too many
              good.replace("CENTER", "CENTRE"),                         # unknown record
              good.replace("\n0\n", "\nfoo\n", 1)):                     # not a number
        with pytest.raises(md.MdockError):
            md.md_autogrid_map_parse(t)


# ------------------------------------------------------------------ rings
def _ring_arrays():
    exp = expected_ligand()
    tp = np.asarray(exp["type_params_from_atom_par_test"], np.float32)
    bonds = np.asarray(exp["bonds"], np.int32)
    tors = [exp["bonds"].index(b) for b in exp["torsion_bonds"]]
    return exp, np.asarray(exp["xyz"], np.float32), np.asarray(exp["types"]), np.asarray(exp["charges"], np.float32), \
        bonds, np.asarray(tors, np.int32), tp


def test_oracle_ring_ligand_moving_sets_and_pairs():
    exp, xyz, types, q, bonds, tors, tp = _ring_arrays()
    ol = OL.prepare(xyz, types, q, bonds, tors, tp, root=0)
    for k, b in enumerate(exp["torsion_bonds"]):
        assert sorted(np.nonzero(ol.moving[k])[0].tolist()) == exp["moving"][f"{b[0]}-{b[1]}"]
    # pairs by hand: ring atoms and the substituents three or more bonds away across C1-C7 or
    # the C7 bonds; nothing inside the ring
    pairs = set(map(tuple, ol.pairs.tolist()))
    ring = set(range(6))
    assert not any(i in ring and j in ring for i, j in pairs)
    assert (1, 6) not in pairs and (0, 7) not in pairs        # C2-C1-C7, C1-C7-O8: two bonds apart
    assert (2, 6) in pairs and (2, 7) in pairs and (0, 8) in pairs and (1, 7) in pairs and (7, 10) in pairs
    assert (7, 9) not in pairs                                 # O8-N10: two bonds apart
    assert (8, 10) in pairs                                    # H9-H11: four bonds, across C7-O8


def test_library_ring_ligand_pairs_equal_oracle():
    exp, xyz, types, q, bonds, tors, tp = _ring_arrays()
    lig = synth.Ligand(xyz, types.astype(np.int32), q, bonds, tors, 0, tp)
    info, slots, _ = md.md_schedule_preview(lig)
    empty = (slots >> 17) & 1
    i, j = slots & 0xFF, (slots >> 8) & 0xFF
    got = sorted(tuple(sorted(p)) for p in zip(i[empty == 0].tolist(), j[empty == 0].tolist()))
    ol = OL.prepare(xyz, types, q, bonds, tors, tp, root=0)
    assert got == sorted(map(tuple, ol.pairs.tolist()))


def test_rotatable_bond_in_a_ring_is_rejected():
    exp, xyz, types, q, bonds, tors, tp = _ring_arrays()
    in_ring = np.asarray([exp["bonds"].index([1, 2])], np.int32)
    with pytest.raises(OL.LigandError):
        OL.prepare(xyz, types, q, bonds, in_ring, tp, root=0)
    with pytest.raises(md.MdockError) as ei:
        md.md_schedule_preview(synth.Ligand(xyz, types.astype(np.int32), q, bonds, in_ring, 0, tp))
    assert "ring" in str(ei.value)
