"""Writes small_dock_oracle.json: the FP64 oracle's complete docks of the small plain workload
(40^3 grid, 20 atoms / 4 rotatable bonds, 1 run x 150 individuals, 10 generations, 6 % local
search x 300 ADADELTA steps) for dock seeds 0..19 -- best genotype, best energy and the best
pose's atom coordinates -- and, for each seed, the same dock on maps perturbed by relative noise
of 1e-7 (about FP32 rounding).  The ADADELTA search is chaotic at this scale (trajectories from
starts 1e-7 apart part ways within a few dozen steps), so the perturbed docks measure how far two
searches that differ only by rounding end up apart: the best-pose RMSD tolerance between the
library and the oracle is set from them.  Calls only oracle/ and workload/.

    python tests/golden/make_small_dock_oracle.py [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "small_dock_oracle.json")
NAME = "plain_fp32_small"
SEEDS = list(range(20))


PERTURB = 1e-7


def dock(args):
    seed, perturbed = args
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import lga as OG
    from oracle import ligand as OL
    from oracle import pose as OP
    from oracle import scoring as S
    from workload import configs
    rec = configs.receptor(NAME)
    lig = configs.ligand(NAME)
    maps = np.asarray(rec.maps, np.float64)
    if perturbed:
        noise = np.random.default_rng([1234, seed]).standard_normal(maps.shape)
        maps = maps * (1.0 + PERTURB * noise)
    grid = S.make_grid(maps, rec.origin, rec.spacing)
    ol = OL.from_synth(lig)
    sp = configs.search_params(NAME, seed=seed)
    keep = {f for f in OG.DockParams.__dataclass_fields__}
    p = OG.DockParams(**{k: v for k, v in sp.items() if k in keep})
    r = OG.lga_dock(grid, ol, p)
    g = np.asarray(r["best_genes"][0], np.float64)
    xyz = OP.pose(ol, g)
    return dict(seed=seed, best_energy=float(r["best_energy"][0]), best_genes=g.tolist(),
                best_xyz=np.asarray(xyz).tolist(), evals=int(r["evals"][0]),
                generations=int(r["generations"][0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    with ProcessPoolExecutor(args.jobs) as ex:
        docks = list(ex.map(dock, [(s, False) for s in SEEDS]))
        perturbed = list(ex.map(dock, [(s, True) for s in SEEDS]))
    out = {"workload": NAME, "what": "FP64 oracle LGA docks (oracle/lga.py lga_dock); best pose per seed",
           "perturbation": f"maps x (1 + {PERTURB} N(0,1)), noise seeded [1234, seed]",
           "docks": docks, "perturbed_docks": perturbed}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: {len(docks)} docks")


if __name__ == "__main__":
    main()
