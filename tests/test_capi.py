"""CPU checks of the C ABI: the library loads, exports every declared entry point, and rejects
malformed input on the host before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mdock.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def md():
    import paper_2203_02096_amd as m
    if not os.path.exists(m.mdock.LIB_PATH):
        from paper_2203_02096_amd import build
        build.build()
    return m


def test_every_declared_symbol_exported(md):
    lib = md.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(md.mdock.SIGNATURES)


def test_one_hip_runtime_in_the_process(md):
    """Loading the library, even before anything imported torch, leaves one HIP runtime in the
    process: torch's, the one whose device buffers and streams the binding passes in.  (With two,
    the second to open the GPU reports that there is no device.)"""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, sys.argv[1]); import paper_2203_02096_amd as m; m.lib(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True, timeout=180,
                         check=True).stdout.strip()
    import ast
    paths = ast.literal_eval(out)
    assert len(paths) == 1, paths


def test_version(md):
    assert b"gfx950" in md.lib().md_version()


def _desc(md, n=6, tors=(), bonds=None, types=None, tp=None):
    from workload import configs
    xyz = np.arange(3 * n, dtype=np.float32).reshape(n, 3)
    bonds = np.array([[i, i + 1] for i in range(n - 1)] if bonds is None else bonds, np.int32).reshape(-1, 2)
    types = np.zeros(n, np.int32) if types is None else np.asarray(types, np.int32)
    tp = configs.type_params() if tp is None else tp
    q = np.zeros(n, np.float32)
    t = np.asarray(tors, np.int32)
    keep = (xyz, bonds, types, tp, q, t)
    d = md.mdock.LigandDesc(n, md.mdock._fptr(xyz), md.mdock._iptr(types), md.mdock._fptr(q),
                            bonds.shape[0], md.mdock._iptr(bonds), t.shape[0], md.mdock._iptr(t), 0,
                            tp.shape[0], md.mdock._fptr(tp))
    return d, keep


@pytest.mark.parametrize("kind,status", [
    ("too_many_atoms", -2), ("not_a_tree", -1), ("terminal_torsion", -1), ("bad_type", -1),
    ("repeat_torsion", -1), ("too_many_torsions", -2), ("zero_atoms", -2),
])
def test_ligand_validation_on_host(md, kind, status):
    lib = md.lib()
    if kind == "too_many_atoms":
        d, keep = _desc(md, n=129)
    elif kind == "zero_atoms":
        d, keep = _desc(md, n=1)
        d.n_atoms = 0
    elif kind == "not_a_tree":
        d, keep = _desc(md, n=6, bonds=[[0, 1], [1, 2], [2, 0], [3, 4], [4, 5]])
    elif kind == "terminal_torsion":
        d, keep = _desc(md, n=6, tors=[0])
    elif kind == "bad_type":
        d, keep = _desc(md, n=6, types=[0, 1, 2, 9, 0, 0])
    elif kind == "repeat_torsion":
        d, keep = _desc(md, n=6, tors=[1, 1])
    else:
        d, keep = _desc(md, n=40, tors=list(range(1, 34)))
    h = C.c_void_p()
    st = lib.md_ligand_create(C.byref(d), C.byref(h))
    assert st == status, lib.md_last_error()
    assert not h.value
    assert lib.md_last_error()


def test_receptor_validation_on_host(md):
    lib = md.lib()
    maps = np.zeros((9, 4, 4, 4), np.float32)
    d = md.mdock.GridDesc(4, 4, 4, 0.375, (C.c_float * 3)(0, 0, 0), 7)
    h = C.c_void_p()
    bad = md.mdock.GridDesc(1, 4, 4, 0.375, (C.c_float * 3)(0, 0, 0), 7)
    assert lib.md_receptor_create(C.byref(bad), md.mdock._fptr(maps), 0, None, C.byref(h)) == -1
    nanmaps = maps.copy()
    nanmaps[3, 1, 1, 1] = np.nan
    assert lib.md_receptor_create(C.byref(d), md.mdock._fptr(nanmaps), 0, None, C.byref(h)) == -1
    big = maps.copy()
    big[0, 0, 0, 0] = 1e6
    assert lib.md_receptor_create(C.byref(d), md.mdock._fptr(big), 1, None, C.byref(h)) == -2
    assert lib.md_receptor_create(C.byref(d), md.mdock._fptr(maps), 7, None, C.byref(h)) == -1
    # cell records of 72 stored values per node must stay below 2 GiB (checked before any map
    # value is read): 196^3 nodes in FP32 and 247^3 in FP16 are past it
    for n, prec in ((196, 0), (247, 1)):
        huge = md.mdock.GridDesc(n, n, n, 0.375, (C.c_float * 3)(0, 0, 0), 7)
        assert lib.md_receptor_create(C.byref(huge), md.mdock._fptr(maps), prec, None, C.byref(h)) == md.mdock.MD_ERANGE
        assert "2 GiB" in lib.md_last_error().decode()
    assert not h.value


def test_null_handles_rejected(md):
    lib = md.lib()
    assert lib.md_eval(None, None, 1, None, None, None, None) == -1
    assert lib.md_local_search(None, None, 1, None, None, None, 10, 0.8, 0.01, None, None) == -1
    assert lib.md_local_search_sw(None, None, 1, None, None, None, 10, 7, None, None) == -1
    assert lib.md_dock(None, None, None, None, None) == -1
    assert lib.md_ligand_num_genes(None) == -1
    plan = md.mdock.Plan(65536, 3, 4, 0, 0, 0)
    assert lib.md_ligand_get_plan(None, C.byref(plan)) == -1
    assert lib.md_ligand_set_plan(None, C.byref(plan)) == -1
    assert lib.md_ligand_autotune(None, None, 0, 0, None, None) == -1
    assert lib.md_schedule_preview(None, C.byref(plan), None, 0, None) == -1
    assert lib.md_server_create(None, None, None) == -1


def test_host_only_settings(md):
    lib = md.lib()
    assert lib.md_tune_table_clear() == 0
    assert lib.md_tune_table_size() == 0
    assert lib.md_graphs_enabled() == 1
    assert lib.md_set_graphs(0) == 0 and lib.md_graphs_enabled() == 0
    assert lib.md_set_graphs(1) == 0 and lib.md_graphs_enabled() == 1


def test_planned_generations_closed_form(md):
    from workload import configs
    p = md.dock_params(**configs.search_params("plain_fp32_small"))
    assert md.md_dock_planned_generations(p) == 10
    p = md.dock_params(**configs.search_params("plain_fp32_production"))
    assert md.md_dock_planned_generations(p) == 56
    # the local optimiser does not change the budget: both spend ls_iters evaluations
    p = md.dock_params(**configs.search_params("plain_fp32_production", ls_method="solis_wets"))
    assert p.ls_method == 1 and md.md_dock_planned_generations(p) == 56
