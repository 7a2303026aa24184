"""The stored cell records of the receptor grid: a single atom of every type placed in the eight
extreme cells of the box and in cells spread through it, evaluated through md_eval against the
oracle's trilinear interpolation of the plain maps (Background: the grid interaction is
interpolated from the eight nodes around an atom).  On a grid with three different axis lengths
a wrong axis stride, corner order or record offset moves an atom onto another cell's values; on
the full-size grids (64^3 FP32 of the production and batched workloads, 96^3 FP16 of the serving
one) the record offsets reach their largest values.  FP16 and BF16 storage are checked against
the oracle on the rounded maps."""
import sys

import numpy as np
import pytest

from oracle import scoring as S
from parity_util import compare, oracle_eval_many, oracle_ligand
from test_gpu_precision import round_maps
from workload import configs, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPACING = 0.375
ORIGIN = (1.5, -2.0, 0.25)
# (nx, ny, nz, storage precision)
GRIDS = [(11, 13, 17, "fp32"), (11, 13, 17, "fp16"), (11, 13, 17, "bf16"), (64, 64, 64, "fp32"), (96, 96, 96, "fp16"),
         (2, 3, 4, "fp32"), (2, 2, 2, "bf16")]   # the smallest grids: one or a few cells, most corners past the end


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


def _maps(nx, ny, nz):
    rng = np.random.default_rng(2203)
    m = rng.normal(0.0, 1.0, size=(synth.N_TYPES + 2, nz, ny, nx)).astype(np.float32)
    m[-1] = np.abs(m[-1])          # desolvation values are not negative
    return m


def _positions(nx, ny, nz):
    """Atom positions: the eight corner cells of the box, then cells drawn through it, each at
    a fractional offset inside its cell away from the faces (where the gradient has kinks)."""
    rng = np.random.default_rng(96)
    cells = [(ix, iy, iz) for ix in (0, nx - 2) for iy in (0, ny - 2) for iz in (0, nz - 2)]
    cells += [tuple(int(rng.integers(0, n - 1)) for n in (nx, ny, nz)) for _ in range(24)]
    pos = []
    for c in cells:
        f = rng.uniform(0.15, 0.85, size=3)
        pos.append(np.asarray(ORIGIN) + (np.asarray(c) + f) * SPACING)
    return np.asarray(pos)


@pytest.mark.parametrize("grid_case", GRIDS, ids=[f"{g[0]}x{g[1]}x{g[2]}-{g[3]}" for g in GRIDS])
def test_single_atoms_in_every_cell_region(md, grid_case):
    nx, ny, nz, precision = grid_case
    maps = _maps(nx, ny, nz)
    drec = md.Receptor(maps, ORIGIN, SPACING, precision)
    stored = maps.astype(np.float64) if precision == "fp32" else round_maps(maps, precision)
    grid = S.make_grid(stored, ORIGIN, SPACING)
    pos = _positions(nx, ny, nz)
    genes = np.zeros((len(pos), 7), np.float32)
    genes[:, 0:3] = pos
    genes[:, 3] = 1.0
    tp = configs.type_params()
    for t in range(synth.N_TYPES):
        lig = synth.Ligand(np.zeros((1, 3), np.float32), np.asarray([t], np.int32), np.asarray([-0.4], np.float32),
                           np.zeros((0, 2), np.int32), np.zeros(0, np.int32), 0, tp)
        dlig = md.Ligand.from_synth(lig)
        g = torch.from_numpy(genes).cuda()
        e = torch.empty(len(genes), device="cuda")
        d = torch.empty(len(genes), 7, device="cuda")
        md.md_eval(drec, dlig, g, e, d)
        torch.cuda.synchronize()
        ref = oracle_eval_many(grid, oracle_ligand(lig), genes)
        stats = compare(ref, e.cpu().numpy(), d.cpu().numpy())
        _say(f"[grid cells] {nx}x{ny}x{nz} {precision} type {t}: {stats}")
        assert stats["checked_energy"] == len(genes) and stats["checked"] == len(genes)
