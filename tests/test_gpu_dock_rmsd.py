"""Best pose of the library's dock against the FP64 oracle's dock of the small plain workload
(40^3 grid, 20 atoms / 4 rotatable bonds, 1 run x 150, 10 generations, 6 % local search x 300
ADADELTA steps), over 20 dock seeds.

Both searches draw the same counter-based random numbers, so they differ only by FP32 versus
FP64 arithmetic.  The search is chaotic at this scale: the oracle itself, run on maps perturbed
by relative noise of 1e-7 (about one FP32 rounding), ends on a different best pose for most
seeds (tests/golden/small_dock_oracle.json holds both sets of oracle docks, written by
tests/golden/make_small_dock_oracle.py).  A bitwise best-pose match is therefore not a property
of the method, and the tolerance is settled on the oracle's own rounding spread:
  * every reported best energy is the oracle's energy of the reported pose (1e-4 rule), and the
    evaluation and generation counts are exact;
  * best-pose RMSD (library vs oracle): the median may be at most twice the median RMSD of the
    perturbed oracle docks (0.90 A, so 1.8 A), and a one-sided Mann-Whitney test may not find the library's RMSDs
    larger than the perturbed ones (p >= 0.01);
  * best energies: the mean of (library - oracle) may not exceed three standard errors of the
    perturbed docks' (perturbed - oracle) spread, in either direction -- the library neither
    docks systematically worse nor differently from a rounding-perturbed oracle."""
import json
import math
import os
import sys

import numpy as np
import pytest

from parity_util import oracle_grid, oracle_ligand
from workload import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "small_dock_oracle.json")
E_TOL = 1e-4
MEDIAN_FACTOR = 2.0
P_MIN = 0.01
SE_FACTOR = 3.0
RMSD_MEDIAN_TOL = 1.8      # Angstrom: twice the perturbed oracle docks' median (0.90 A), rounded up


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rmsd(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.sqrt(np.mean(np.sum((a - b) ** 2, axis=1))))


def test_small_dock_best_pose_within_rounding_spread():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from scipy import stats

    import paper_2203_02096_amd as md
    from oracle import scoring as S
    golden = json.load(open(GOLDEN))
    name = golden["workload"]
    rec = configs.receptor(name)
    lig = configs.ligand(name)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing)
    dlig = md.Ligand.from_synth(lig)
    grid, ol = oracle_grid(rec), oracle_ligand(lig)
    r_gpu, r_pert, d_gpu, d_pert = [], [], [], []
    for d, p in zip(golden["docks"], golden["perturbed_docks"]):
        assert d["seed"] == p["seed"]
        res = md.md_dock(drec, dlig, md.dock_params(**configs.search_params(name, seed=d["seed"])))
        assert int(res["evals"][0]) == d["evals"] and int(res["generations"][0]) == d["generations"]
        e_gpu = float(res["best_energy"][0])
        ref = S.energy_and_gradient(grid, ol, res["best_genes"][0].astype(np.float64))
        assert abs(ref.energy - e_gpu) <= E_TOL * max(abs(ref.energy), ref.scale_energy)
        r_gpu.append(_rmsd(res["best_xyz"][0], d["best_xyz"]))
        r_pert.append(_rmsd(p["best_xyz"], d["best_xyz"]))
        d_gpu.append(e_gpu - d["best_energy"])
        d_pert.append(p["best_energy"] - d["best_energy"])
        _say(f"[best pose] seed {d['seed']:2d}: RMSD lib {r_gpu[-1]:.3f} A (perturbed oracle {r_pert[-1]:.3f}); "
             f"E lib {e_gpu:.4f} oracle {d['best_energy']:.4f} perturbed {p['best_energy']:.4f}")
    med_gpu, med_pert = float(np.median(r_gpu)), float(np.median(r_pert))
    pval = float(stats.mannwhitneyu(r_gpu, r_pert, alternative="greater").pvalue)
    bound = SE_FACTOR * float(np.std(d_pert, ddof=1)) / math.sqrt(len(d_pert))
    _say(f"[best pose] median RMSD lib {med_gpu:.3f} A, perturbed oracle {med_pert:.3f} A, "
         f"Mann-Whitney p {pval:.3f}; mean dE lib {np.mean(d_gpu):+.3f}, perturbed {np.mean(d_pert):+.3f}, "
         f"bound +-{bound:.3f} kcal/mol")
    assert med_gpu <= MEDIAN_FACTOR * med_pert and med_gpu <= RMSD_MEDIAN_TOL
    assert pval >= P_MIN
    assert abs(float(np.mean(d_gpu))) <= bound
