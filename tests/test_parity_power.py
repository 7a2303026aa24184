"""The GPU parity rule can see a wrong grid term: mistakes planted in the oracle's grid term, on
the CPU, fail the comparison on the clean poses that the GPU eval-parity tests use.

The tolerance (1e-4 of the larger of |E| and the sum of |terms|) is relative to the whole pose,
so on clashing or out-of-grid poses it can exceed the whole grid term; the clean-pose sampler
exists so that it does not.  Each planted mistake is one that a kernel could plausibly make: the
grid term of the second atom slot per lane (atoms 64 and up) lost, the electrostatic map's sign
flipped, the desolvation map weighted by q instead of |q|, and the type maps read at a corner
one node over along x."""
import numpy as np
import pytest

from parity_util import E_TOL, KINK, clean_genes, oracle_eval_many, oracle_grid, oracle_ligand
from oracle import constants as C
from oracle import scoring as S
from workload import configs, synth

CASES = [("production_40a_8t", 64, 102, 40, 8, 202, 24), ("edge_65a_12t", 64, 102, 65, 12, 306, 16),
         ("wide_100a_32t", 64, 102, 100, 32, 303, 12), ("max_128a_32t", 64, 102, 128, 32, 304, 10)]


def _grid_terms(grid, r, ol, mutate):
    """Per-atom grid energies of pose r under the planted mistake `mutate`."""
    x = r.x
    if mutate == "shift_x":
        g = S.Grid(maps=np.roll(grid.maps, -1, axis=3), origin=grid.origin, spacing=grid.spacing)
        return S.grid_energies(g, x, ol.types, ol.charges)[0]
    if mutate == "elec_sign":
        return _split(grid, x, ol, elec=-1.0)
    if mutate == "desolv_q":
        return _split(grid, x, ol, desolv_signed=True)
    e = S.grid_energies(grid, x, ol.types, ol.charges)[0].copy()
    if mutate == "drop_slot2":
        e[64:] = 0.0
    return e


def _split(grid, x, ol, elec=1.0, desolv_signed=False):
    """Grid energies with the electrostatic term scaled by `elec` and the desolvation map
    weighted by q instead of |q| when desolv_signed."""
    ins, g = S.inside(grid, x)
    ins = np.atleast_1d(ins)
    q = np.asarray(ol.charges, np.float64)
    e = S.grid_energies(grid, x, ol.types, ol.charges)[0].copy()
    if np.any(ins):
        ve, _ = S.trilinear(grid.maps[C.N_TYPES], g[ins])
        vd, _ = S.trilinear(grid.maps[C.N_TYPES + 1], g[ins])
        e[ins] += (elec - 1.0) * q[ins] * ve
        if desolv_signed:
            e[ins] += (q[ins] - np.abs(q[ins])) * vd
    return e


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mutate", ["drop_slot2", "elec_sign", "desolv_q", "shift_x"])
def test_planted_grid_mistakes_fail_the_rule(case, mutate):
    name, gn, ms, na, nt, ls, npose = case
    if mutate == "drop_slot2" and na <= 64:
        pytest.skip("one atom slot per lane")
    rec = synth.make_receptor(gn, ms)
    lig = synth.make_ligand(na, nt, ls, configs.type_params())
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    genes, _ = clean_genes(lig, rec, npose, seed=ls, olig=ol, grid=grid)
    refs = oracle_eval_many(grid, ol, genes)
    caught = checked = 0
    for r in refs:
        if r.margin_energy < KINK:     # the GPU comparison skips these too
            continue
        e_true = S.grid_energies(grid, r.x, ol.types, ol.charges)[0]
        e_bad = r.energy - float(e_true.sum()) + float(_grid_terms(grid, r, ol, mutate).sum())
        tol = E_TOL * max(abs(r.energy), r.scale_energy)
        checked += 1
        caught += abs(e_bad - r.energy) > tol
    assert checked >= 0.8 * npose
    assert caught >= 0.9 * checked, (mutate, caught, checked)
