"""Thin Python binding of libmdock (include/mdock.h): argument marshalling only.

Device buffers are torch CUDA (HIP) tensors; streams are torch streams.  Every step of
the docking path runs in the library's HIP kernels; nothing here computes.  If
libmdock.so has not been built the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdock.so")

MD_OK, MD_EINVAL, MD_ERANGE, MD_ENOMEM, MD_EDEVICE = 0, -1, -2, -3, -4
PRECISION = {"fp32": 0, "fp16": 1, "bf16": 2}

_lib = None


class MdockError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmdock status {status}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("spacing", C.c_float),
                ("origin", C.c_float * 3), ("n_types", C.c_int)]


class LigandDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("xyz", C.POINTER(C.c_float)), ("type", C.POINTER(C.c_int)),
                ("charge", C.POINTER(C.c_float)), ("n_bonds", C.c_int), ("bonds", C.POINTER(C.c_int)),
                ("n_torsions", C.c_int), ("torsions", C.POINTER(C.c_int)), ("root_atom", C.c_int),
                ("n_types", C.c_int), ("type_params", C.POINTER(C.c_float))]


class PdbqtLigand(C.Structure):
    _fields_ = [("max_atoms", C.c_int), ("max_bonds", C.c_int), ("max_torsions", C.c_int),
                ("n_atoms", C.c_int), ("n_bonds", C.c_int), ("n_torsions", C.c_int), ("root_atom", C.c_int),
                ("xyz", C.POINTER(C.c_float)), ("charge", C.POINTER(C.c_float)), ("type", C.POINTER(C.c_int)),
                ("bonds", C.POINTER(C.c_int)), ("torsions", C.POINTER(C.c_int)), ("serial", C.POINTER(C.c_int))]


class DockParams(C.Structure):
    _fields_ = [("n_runs", C.c_int), ("pop_size", C.c_int), ("max_evals_per_run", C.c_longlong),
                ("max_generations", C.c_int), ("ls_rate", C.c_float), ("ls_iters", C.c_int),
                ("rho", C.c_float), ("eps", C.c_float), ("crossover_rate", C.c_float),
                ("mutation_rate", C.c_float), ("tournament_rate", C.c_float), ("elitism", C.c_int),
                ("mut_trans", C.c_float), ("mut_rot", C.c_float), ("mut_tors", C.c_float),
                ("seed", C.c_ulonglong), ("ls_method", C.c_int)]


LS_METHODS = {"adadelta": 0, "solis_wets": 1}


class DockResult(C.Structure):
    _fields_ = [("n_runs", C.c_int), ("n_genes", C.c_int), ("n_atoms", C.c_int),
                ("best_energy", C.POINTER(C.c_float)), ("best_genes", C.POINTER(C.c_float)),
                ("best_xyz", C.POINTER(C.c_float)), ("run_index", C.POINTER(C.c_int)),
                ("evals", C.POINTER(C.c_longlong)), ("generations", C.POINTER(C.c_int))]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int), ("use_graphs", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("ticks", C.c_longlong), ("completed", C.c_longlong), ("queued", C.c_int),
                ("resident", C.c_int), ("pool_used_bytes", C.c_size_t), ("busy_seconds", C.c_double)]


class Plan(C.Structure):
    _fields_ = [("lds_budget", C.c_int), ("group_div", C.c_int), ("waves_per_block", C.c_int),
                ("lds_bytes", C.c_int), ("staged_rows", C.c_int), ("total_rows", C.c_int),
                ("waves_per_pose", C.c_int)]


class TuneInfo(C.Structure):
    _fields_ = [("plan", Plan), ("us_per_eval", C.c_double), ("default_us_per_eval", C.c_double),
                ("candidates", C.c_int), ("from_table", C.c_int)]


class BatchTuneInfo(C.Structure):
    _fields_ = [("policy", C.c_int), ("n_policies", C.c_int), ("ms_per_generation", C.c_double * 8)]


BATCH_POLICIES = ["default", "tuned_alone", "lds_all", "wide_blocks", "small_groups", "shared_large", "full_blocks"]


class DockJob(C.Structure):
    _fields_ = [("ligand", C.c_void_p), ("params", DockParams), ("result", C.POINTER(DockResult))]


# name -> (restype, argtypes); the complete exported surface of include/mdock.h
SIGNATURES = {
    "md_autogrid_map_parse": (C.c_int, [C.c_char_p, C.c_longlong, C.c_void_p, C.c_void_p, C.c_longlong,
                                        C.POINTER(C.c_longlong)]),
    "md_pdbqt_parse": (C.c_int, [C.c_char_p, C.c_longlong, C.c_int, C.POINTER(C.c_char_p), C.c_void_p]),
    "md_atom_par_parse": (C.c_int, [C.c_char_p, C.c_longlong, C.c_int, C.POINTER(C.c_char_p), C.c_void_p]),
    "md_receptor_create": (C.c_int, [C.POINTER(GridDesc), C.POINTER(C.c_float), C.c_int, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "md_receptor_destroy": (C.c_int, [C.c_void_p]),
    "md_ligand_create": (C.c_int, [C.POINTER(LigandDesc), C.POINTER(C.c_void_p)]),
    "md_ligand_destroy": (C.c_int, [C.c_void_p]),
    "md_ligand_num_genes": (C.c_int, [C.c_void_p]),
    "md_ligand_num_atoms": (C.c_int, [C.c_void_p]),
    "md_ligand_num_pairs": (C.c_int, [C.c_void_p]),
    "md_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "md_pose": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "md_local_search": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int, C.c_float, C.c_float, C.c_void_p, C.c_void_p]),
    "md_local_search_sw": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int, C.c_ulonglong, C.c_void_p, C.c_void_p]),
    "md_local_search_traced": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_int, C.c_float, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "md_dock": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(DockParams), C.POINTER(DockResult), C.c_void_p]),
    "md_dock_batch": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(DockJob), C.c_void_p]),
    "md_dock_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(DockParams), C.POINTER(DockResult), C.c_void_p]),
    "md_dock_planned_generations": (C.c_int, [C.POINTER(DockParams)]),
    "md_server_create": (C.c_int, [C.c_void_p, C.POINTER(ServerParams), C.POINTER(C.c_void_p)]),
    "md_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(DockParams), C.POINTER(C.c_ulonglong)]),
    "md_server_poll": (C.c_int, [C.c_void_p, C.c_ulonglong, C.POINTER(DockResult), C.POINTER(C.c_int)]),
    "md_server_wait": (C.c_int, [C.c_void_p, C.c_ulonglong, C.POINTER(DockResult), C.c_double]),
    "md_server_cancel": (C.c_int, [C.c_void_p, C.c_ulonglong]),
    "md_server_request_times": (C.c_int, [C.c_void_p, C.c_ulonglong, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "md_server_release": (C.c_int, [C.c_void_p, C.c_ulonglong]),
    "md_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "md_server_destroy": (C.c_int, [C.c_void_p]),
    "md_ligand_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)]),
    "md_profile_enable": (C.c_int, [C.c_int]),
    "md_profile_reset": (C.c_int, []),
    "md_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "md_set_graphs": (C.c_int, [C.c_int]),
    "md_ligand_get_plan": (C.c_int, [C.c_void_p, C.POINTER(Plan)]),
    "md_ligand_set_plan": (C.c_int, [C.c_void_p, C.POINTER(Plan)]),
    "md_ligand_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(TuneInfo)]),
    "md_tune_table_clear": (C.c_int, []),
    "md_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p), C.POINTER(DockParams), C.c_int,
                                    C.c_void_p, C.POINTER(BatchTuneInfo)]),
    "md_schedule_preview": (C.c_int, [C.POINTER(LigandDesc), C.POINTER(Plan), C.POINTER(C.c_uint), C.c_int,
                                      C.POINTER(C.c_int)]),
    "md_tune_table_size": (C.c_int, []),
    "md_graphs_enabled": (C.c_int, []),
    "md_last_error": (C.c_char_p, []),
    "md_version": (C.c_char_p, []),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_02096_amd.build`")
        # torch brings its own copy of the HIP runtime, and the device buffers and streams passed
        # to the library are torch's: torch is loaded first so that the library binds to that
        # copy.  Loaded the other way round, the process holds two HIP runtimes and the second
        # one to open the GPU finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, what):
    if status != MD_OK:
        raise MdockError(status, lib().md_last_error().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name, shape=None, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class Receptor:
    """Grid maps on the device (md_receptor_create)."""

    def __init__(self, maps, origin, spacing, precision="fp32", stream=None):
        maps = np.ascontiguousarray(maps, dtype=np.float32)
        if maps.ndim != 4:
            raise ValueError("maps must be [n_types+2][nz][ny][nx]")
        nm, nz, ny, nx = maps.shape
        d = GridDesc(nx, ny, nz, float(spacing), (C.c_float * 3)(*[float(v) for v in origin]), nm - 2)
        h = C.c_void_p()
        self._maps_ref = maps
        _check(lib().md_receptor_create(C.byref(d), _fptr(maps), PRECISION[precision],
                                        _stream_ptr(stream) if stream is not False else None, C.byref(h)),
               "md_receptor_create")
        self.handle = h
        self.shape = (nx, ny, nz)
        self.precision = precision

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.md_receptor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ligand:
    """Preprocessed ligand on the device (md_ligand_create)."""

    def __init__(self, xyz, types, charges, bonds, torsions, type_params, root=0):
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        self._types = np.ascontiguousarray(types, dtype=np.int32).reshape(-1)
        self._q = np.ascontiguousarray(charges, dtype=np.float32).reshape(-1)
        self._bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
        self._tors = np.ascontiguousarray(torsions, dtype=np.int32).reshape(-1)
        self._tp = np.ascontiguousarray(type_params, dtype=np.float32).reshape(-1, 7)
        d = LigandDesc(self._xyz.shape[0], _fptr(self._xyz), _iptr(self._types), _fptr(self._q),
                       self._bonds.shape[0], _iptr(self._bonds), self._tors.shape[0], _iptr(self._tors),
                       int(root), self._tp.shape[0], _fptr(self._tp))
        h = C.c_void_p()
        _check(lib().md_ligand_create(C.byref(d), C.byref(h)), "md_ligand_create")
        self.handle = h
        self.n_genes = lib().md_ligand_num_genes(h)
        self.n_atoms = lib().md_ligand_num_atoms(h)
        self.n_pairs = lib().md_ligand_num_pairs(h)

    @classmethod
    def from_synth(cls, lig):
        return cls(lig.xyz, lig.types, lig.charges, lig.bonds, lig.torsions, lig.type_params,
                   getattr(lig, "root", 0))

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.md_ligand_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _text(t):
    return t.encode() if isinstance(t, str) else bytes(t)


def _names(type_names):
    arr = (C.c_char_p * len(type_names))(*[n.encode() for n in type_names])
    return arr


def md_autogrid_map_parse(text):
    """One AutoGrid map file's text -> (desc dict, values float32 [nz][ny][nx])."""
    b = _text(text)
    d = GridDesc()
    n = C.c_longlong()
    _check(lib().md_autogrid_map_parse(b, len(b), C.byref(d), None, 0, C.byref(n)), "md_autogrid_map_parse")
    vals = np.zeros(n.value, np.float32)
    _check(lib().md_autogrid_map_parse(b, len(b), C.byref(d), _fptr(vals), vals.size, C.byref(n)),
           "md_autogrid_map_parse")
    desc = dict(shape=(d.nx, d.ny, d.nz), spacing=d.spacing, origin=tuple(d.origin))
    return desc, vals.reshape(d.nz, d.ny, d.nx)


def md_pdbqt_parse(text, type_names, max_atoms=256, max_bonds=1024, max_torsions=64):
    """A PDBQT ligand's text -> dict of xyz, charges, types (indices into type_names), bonds,
    torsions (indices into bonds), root, serial."""
    b = _text(text)
    names = _names(type_names)
    out = dict(xyz=np.zeros((max_atoms, 3), np.float32), charges=np.zeros(max_atoms, np.float32),
               types=np.zeros(max_atoms, np.int32), bonds=np.zeros((max_bonds, 2), np.int32),
               torsions=np.zeros(max_torsions, np.int32), serial=np.zeros(max_atoms, np.int32))
    r = PdbqtLigand(max_atoms, max_bonds, max_torsions, 0, 0, 0, 0, _fptr(out["xyz"]), _fptr(out["charges"]),
                    _iptr(out["types"]), _iptr(out["bonds"]), _iptr(out["torsions"]), _iptr(out["serial"]))
    _check(lib().md_pdbqt_parse(b, len(b), len(type_names), names, C.byref(r)), "md_pdbqt_parse")
    n, nb, nt = r.n_atoms, r.n_bonds, r.n_torsions
    return dict(xyz=out["xyz"][:n].copy(), charges=out["charges"][:n].copy(), types=out["types"][:n].copy(),
                bonds=out["bonds"][:nb].copy(), torsions=out["torsions"][:nt].copy(), root=r.root_atom,
                serial=out["serial"][:n].copy())


def md_atom_par_parse(text, type_names):
    """atom_par records -> type_params float32 [len(type_names)][7]."""
    b = _text(text)
    tp = np.zeros((len(type_names), 7), np.float32)
    _check(lib().md_atom_par_parse(b, len(b), len(type_names), _names(type_names), _fptr(tp)),
           "md_atom_par_parse")
    return tp


def receptor_from_autogrid(map_texts, precision="fp32", stream=None):
    """Nine AutoGrid map texts of one grid (the seven type maps in type order, then the
    electrostatic and the desolvation map) -> Receptor."""
    if len(map_texts) != 9:
        raise ValueError("a receptor is 7 type maps, the electrostatic map and the desolvation map")
    descs, vals = zip(*[md_autogrid_map_parse(t) for t in map_texts])
    if any(d != descs[0] for d in descs):
        raise ValueError("the maps do not share one grid")
    return Receptor(np.stack(vals), descs[0]["origin"], descs[0]["spacing"], precision, stream)


def ligand_from_pdbqt(text, type_names, type_params):
    """A PDBQT ligand whose atom types index the receptor's seven type maps (type_names), with
    the type parameters of those types -> Ligand."""
    p = md_pdbqt_parse(text, type_names)
    return Ligand(p["xyz"], p["types"], p["charges"], p["bonds"], p["torsions"], type_params, p["root"])


def md_eval(rec: Receptor, lig: Ligand, genes, energy, grad=None, stream=None):
    import torch
    n = genes.shape[0] if genes.ndim == 2 else 0
    gp = _dev_ptr(genes, "genes", (n, lig.n_genes), torch.float32)
    ep = _dev_ptr(energy, "energy", (n,), torch.float32)
    dp = _dev_ptr(grad, "grad", (n, lig.n_genes), torch.float32) if grad is not None else None
    _check(lib().md_eval(rec.handle, lig.handle, n, gp, ep, dp, _stream_ptr(stream)), "md_eval")


def md_pose(lig: Ligand, genes, xyz, stream=None):
    import torch
    n = genes.shape[0]
    _check(lib().md_pose(lig.handle, n, _dev_ptr(genes, "genes", (n, lig.n_genes), torch.float32),
                         _dev_ptr(xyz, "xyz", (n, lig.n_atoms, 3), torch.float32), _stream_ptr(stream)),
           "md_pose")


def md_local_search(rec: Receptor, lig: Ligand, genes_in, genes_out, energy_out, n_iters=300,
                    rho=0.8, eps=1e-2, trace=None, stream=None):
    import torch
    n = genes_in.shape[0]
    tp = _dev_ptr(trace, "trace", (n, n_iters), torch.float32) if trace is not None else None
    _check(lib().md_local_search(rec.handle, lig.handle, n,
                                 _dev_ptr(genes_in, "genes_in", (n, lig.n_genes), torch.float32),
                                 _dev_ptr(genes_out, "genes_out", (n, lig.n_genes), torch.float32),
                                 _dev_ptr(energy_out, "energy_out", (n,), torch.float32),
                                 int(n_iters), float(rho), float(eps), tp, _stream_ptr(stream)),
           "md_local_search")


def md_local_search_traced(rec: Receptor, lig: Ligand, genes_in, genes_out, energy_out, n_iters=300,
                           rho=0.8, eps=1e-2, trace=None, trace_genes=None, trace_grad=None, stream=None):
    """md_local_search that also records each step's iterate and gradient ([n][n_iters][n_genes])."""
    import torch
    n = genes_in.shape[0]
    G = lig.n_genes
    tp = _dev_ptr(trace, "trace", (n, n_iters), torch.float32) if trace is not None else None
    tx = _dev_ptr(trace_genes, "trace_genes", (n, n_iters, G), torch.float32) if trace_genes is not None else None
    tg = _dev_ptr(trace_grad, "trace_grad", (n, n_iters, G), torch.float32) if trace_grad is not None else None
    _check(lib().md_local_search_traced(rec.handle, lig.handle, n,
                                        _dev_ptr(genes_in, "genes_in", (n, G), torch.float32),
                                        _dev_ptr(genes_out, "genes_out", (n, G), torch.float32),
                                        _dev_ptr(energy_out, "energy_out", (n,), torch.float32),
                                        int(n_iters), float(rho), float(eps), tp, tx, tg, _stream_ptr(stream)),
           "md_local_search_traced")


def md_local_search_sw(rec: Receptor, lig: Ligand, genes_in, genes_out, energy_out, n_evals=300,
                       seed=7, trace=None, stream=None):
    import torch
    n = genes_in.shape[0]
    tp = _dev_ptr(trace, "trace", (n, n_evals), torch.float32) if trace is not None else None
    _check(lib().md_local_search_sw(rec.handle, lig.handle, n,
                                    _dev_ptr(genes_in, "genes_in", (n, lig.n_genes), torch.float32),
                                    _dev_ptr(genes_out, "genes_out", (n, lig.n_genes), torch.float32),
                                    _dev_ptr(energy_out, "energy_out", (n,), torch.float32),
                                    int(n_evals), int(seed), tp, _stream_ptr(stream)),
           "md_local_search_sw")


def dock_params(**kw) -> DockParams:
    """md_dock_params with the library's defaults; ls_method may be given by name."""
    p = DockParams()
    defaults = dict(n_runs=1, pop_size=150, max_evals_per_run=2_500_000, max_generations=27000,
                    ls_rate=0.06, ls_iters=300, rho=0.8, eps=1e-2, crossover_rate=0.8,
                    mutation_rate=0.02, tournament_rate=0.6, elitism=1, mut_trans=2.0,
                    mut_rot=float(np.pi / 2), mut_tors=float(np.pi), seed=7, ls_method=0)
    defaults.update(kw)
    if isinstance(defaults["ls_method"], str):
        defaults["ls_method"] = LS_METHODS[defaults["ls_method"]]
    for k, v in defaults.items():
        setattr(p, k, v)
    return p


def md_dock_planned_generations(params: DockParams) -> int:
    return lib().md_dock_planned_generations(C.byref(params))


def _result(params, lig, want_xyz):
    R, G, N = params.n_runs, lig.n_genes, lig.n_atoms
    arrs = dict(best_energy=np.zeros(R, np.float32), best_genes=np.zeros((R, G), np.float32),
                best_xyz=np.zeros((R, N, 3), np.float32) if want_xyz else None,
                run_index=np.zeros(R, np.int32), evals=np.zeros(R, np.int64),
                generations=np.zeros(R, np.int32))
    res = DockResult(R, G, N, _fptr(arrs["best_energy"]), _fptr(arrs["best_genes"]),
                     _fptr(arrs["best_xyz"]) if want_xyz else None, _iptr(arrs["run_index"]),
                     arrs["evals"].ctypes.data_as(C.POINTER(C.c_longlong)), _iptr(arrs["generations"]))
    return res, arrs


def md_dock(rec: Receptor, lig: Ligand, params: DockParams, stream=None, want_xyz=True):
    res, arrs = _result(params, lig, want_xyz)
    _check(lib().md_dock(rec.handle, lig.handle, C.byref(params), C.byref(res), _stream_ptr(stream)),
           "md_dock")
    return arrs


def md_dock_noalloc(rec: Receptor, lig: Ligand, params: DockParams, stream=None, want_xyz=True):
    """md_dock with its workspace in the library's static device array (no device allocation)."""
    res, arrs = _result(params, lig, want_xyz)
    _check(lib().md_dock_noalloc(rec.handle, lig.handle, C.byref(params), C.byref(res), _stream_ptr(stream)),
           "md_dock_noalloc")
    return arrs


def md_dock_batch(rec: Receptor, jobs, stream=None, want_xyz=True):
    """jobs: sequence of (Ligand, DockParams); returns one result dict per job."""
    jobs = list(jobs)
    keep, out = [], []
    arr = (DockJob * max(1, len(jobs)))()
    for k, (lig, params) in enumerate(jobs):
        res, arrs = _result(params, lig, want_xyz)
        keep.append(res)
        out.append(arrs)
        arr[k].ligand = lig.handle
        arr[k].params = params
        arr[k].result = C.pointer(res)
    _check(lib().md_dock_batch(rec.handle, len(jobs), arr, _stream_ptr(stream)), "md_dock_batch")
    return out


KERNELS = {"init_population": 0, "generation": 1, "ls_pick": 2, "local_search": 3, "sum_evals": 4,
           "best_of_runs": 5}


def md_ligand_info(lig: Ligand):
    v = [C.c_int() for _ in range(4)]
    _check(lib().md_ligand_info(lig.handle, *[C.byref(x) for x in v]), "md_ligand_info")
    return dict(n_atoms=v[0].value, n_torsions=v[1].value, n_pairs=v[2].value, sum_moving=v[3].value)


def md_profile_enable(on=True):
    _check(lib().md_profile_enable(int(bool(on))), "md_profile_enable")


def md_profile_reset():
    _check(lib().md_profile_reset(), "md_profile_reset")


def _plan_dict(p: Plan):
    return {k: getattr(p, k) for k, _ in Plan._fields_}


def md_ligand_get_plan(lig: Ligand):
    p = Plan()
    _check(lib().md_ligand_get_plan(lig.handle, C.byref(p)), "md_ligand_get_plan")
    return _plan_dict(p)


def md_ligand_set_plan(lig: Ligand, lds_budget=65536, group_div=3, waves_per_block=4, waves_per_pose=1):
    p = Plan(int(lds_budget), int(group_div), int(waves_per_block), 0, 0, 0, int(waves_per_pose))
    _check(lib().md_ligand_set_plan(lig.handle, C.byref(p)), "md_ligand_set_plan")
    return md_ligand_get_plan(lig)


def md_ligand_autotune(rec: Receptor, lig: Ligand, n_starts=0, force=False, stream=None):
    """Times candidate launch plans of the ligand on this receptor for launches of n_starts local
    searches (0: launches that fill the device) and keeps the fastest."""
    info = TuneInfo()
    _check(lib().md_ligand_autotune(rec.handle, lig.handle, int(n_starts), 1 if force else 0,
                                    _stream_ptr(stream), C.byref(info)), "md_ligand_autotune")
    return dict(plan=_plan_dict(info.plan), us_per_eval=info.us_per_eval,
                default_us_per_eval=info.default_us_per_eval, candidates=info.candidates,
                from_table=bool(info.from_table))


def md_schedule_preview(lig, lds_budget=65536, group_div=3, waves_per_block=4, waves_per_pose=1):
    """Host only: the pair schedule (slots i | j<<8 | hb<<16 | empty<<17, row-major) that a plan
    gives a ligand described like workload.synth.Ligand; returns (plan dict, slots, group_lanes)."""
    xyz = np.ascontiguousarray(lig.xyz, dtype=np.float32).reshape(-1, 3)
    types = np.ascontiguousarray(lig.types, dtype=np.int32).reshape(-1)
    q = np.ascontiguousarray(lig.charges, dtype=np.float32).reshape(-1)
    bonds = np.ascontiguousarray(lig.bonds, dtype=np.int32).reshape(-1, 2)
    tors = np.ascontiguousarray(lig.torsions, dtype=np.int32).reshape(-1)
    tp = np.ascontiguousarray(lig.type_params, dtype=np.float32).reshape(-1, 7)
    d = LigandDesc(xyz.shape[0], _fptr(xyz), _iptr(types), _fptr(q), bonds.shape[0], _iptr(bonds),
                   tors.shape[0], _iptr(tors), int(getattr(lig, "root", 0)), tp.shape[0], _fptr(tp))
    p = Plan(int(lds_budget), int(group_div), int(waves_per_block), 0, 0, 0, int(waves_per_pose))
    gl = C.c_int()
    _check(lib().md_schedule_preview(C.byref(d), C.byref(p), None, 0, C.byref(gl)), "md_schedule_preview")
    slots = np.zeros(p.total_rows * 64, dtype=np.uint32)
    p2 = Plan(int(lds_budget), int(group_div), int(waves_per_block), 0, 0, 0, int(waves_per_pose))
    _check(lib().md_schedule_preview(C.byref(d), C.byref(p2), slots.ctypes.data_as(C.POINTER(C.c_uint)),
                                     slots.size, C.byref(gl)), "md_schedule_preview")
    return _plan_dict(p2), slots, gl.value


def md_batch_autotune(rec: Receptor, jobs, generations=6, stream=None):
    """Times whole-batch launch-plan policies on the batch itself (jobs: (Ligand, DockParams)
    pairs, run to generations/3 and to `generations` generations) and applies the fastest to
    every ligand."""
    jobs = list(jobs)
    ligs = (C.c_void_p * len(jobs))(*[l.handle.value for l, _ in jobs])
    params = (DockParams * len(jobs))(*[p for _, p in jobs])
    info = BatchTuneInfo()
    _check(lib().md_batch_autotune(rec.handle, len(jobs), ligs, params, int(generations), _stream_ptr(stream),
                                   C.byref(info)), "md_batch_autotune")
    return dict(policy=BATCH_POLICIES[info.policy],
                ms_per_generation={BATCH_POLICIES[k]: info.ms_per_generation[k] for k in range(info.n_policies)})


def md_tune_table_clear():
    _check(lib().md_tune_table_clear(), "md_tune_table_clear")


def md_tune_table_size():
    return int(lib().md_tune_table_size())


def md_set_graphs(on=True):
    """Capture and replay each LGA generation as a HIP graph (default on)."""
    _check(lib().md_set_graphs(int(bool(on))), "md_set_graphs")


def md_graphs_enabled():
    return bool(lib().md_graphs_enabled())


def md_profile_read(kind):
    ms, n = C.c_double(), C.c_longlong()
    _check(lib().md_profile_read(KERNELS.get(kind, kind), C.byref(ms), C.byref(n)), "md_profile_read")
    return ms.value, n.value


class Server:
    """Continuous-batching docking server (md_server_*).  Keep the receptor and every submitted
    Ligand alive while the server runs."""

    def __init__(self, rec: Receptor, hbm_budget_bytes=1 << 30, max_slots=64, use_graphs=True):
        h = C.c_void_p()
        p = ServerParams(int(hbm_budget_bytes), int(max_slots), int(bool(use_graphs)))
        _check(lib().md_server_create(rec.handle, C.byref(p), C.byref(h)), "md_server_create")
        self.handle = h
        self._rec = rec
        self._ligs = {}

    def submit(self, lig: Ligand, params: DockParams) -> int:
        t = C.c_ulonglong()
        _check(lib().md_server_submit(self.handle, lig.handle, C.byref(params), C.byref(t)), "md_server_submit")
        self._ligs[t.value] = (lig, params)
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0, want_xyz=True):
        lig, params = self._ligs[ticket]
        res, arrs = _result(params, lig, want_xyz)
        _check(lib().md_server_wait(self.handle, ticket, C.byref(res), float(timeout_s)), "md_server_wait")
        return arrs

    def poll(self, ticket: int, want_xyz=True):
        lig, params = self._ligs[ticket]
        res, arrs = _result(params, lig, want_xyz)
        done = C.c_int()
        _check(lib().md_server_poll(self.handle, ticket, C.byref(res), C.byref(done)), "md_server_poll")
        return arrs if done.value else None

    def cancel(self, ticket: int):
        _check(lib().md_server_cancel(self.handle, ticket), "md_server_cancel")

    def times(self, ticket: int):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().md_server_request_times(self.handle, ticket, C.byref(a), C.byref(b), C.byref(c)),
               "md_server_request_times")
        return a.value, b.value, c.value

    def release(self, ticket: int):
        _check(lib().md_server_release(self.handle, ticket), "md_server_release")
        self._ligs.pop(ticket, None)

    def stats(self):
        st = ServerStats()
        _check(lib().md_server_get_stats(self.handle, C.byref(st)), "md_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.md_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
