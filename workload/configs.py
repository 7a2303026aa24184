"""Named synthetic workloads (sizes and seeds only; no method arithmetic).

plain_fp32_small      40^3 grid, one ligand of 20 atoms / 4 rotatable bonds,
                      1 run x 150 individuals, 10 generations, 6 % local search x 300
                      ADADELTA steps.  Small enough for the oracle to dock in seconds.
plain_fp32_production 64^3 grid, one ligand of 40 atoms / 8 rotatable bonds,
                      20 runs x 150, 2.5M energy evaluations per run, local search
                      on every individual.
batched_fp32          one 64^3 map set, 256 ligands (10-100 atoms, 0-32 rotatable
                      bonds), 10 runs x 150 each.
serving_fp16          96^3 map set, ligands of log-normal size (median 35, 10-120
                      atoms), 10 runs x 150, 250k evaluations per run.
paper_inputs          the paper's three input sizes (small / medium / large ligands of 21, 43
                      and 108 atoms with 2, 15 and 31 rotatable bonds; Background, "Design and
                      Structure of MiniMDock") as synthetic ligands on the 64^3 map set, run
                      with 10 and 100 runs (its threads-per-workgroup study, Section "Results"),
                      2.5M evaluations per run, 6 % local search x 300.
"""
from __future__ import annotations

import math

import numpy as np

from . import synth

TYPE_SEED = 1234

WORKLOADS = {
    "plain_fp32_small": dict(grid=40, map_seed=101, n_atoms=20, n_torsions=4, lig_seed=201,
                             n_runs=1, pop_size=150, max_generations=10,
                             max_evals_per_run=10**12, ls_rate=0.06, ls_iters=300),
    "plain_fp32_production": dict(grid=64, map_seed=102, n_atoms=40, n_torsions=8, lig_seed=202,
                                  n_runs=20, pop_size=150, max_generations=10**6,
                                  max_evals_per_run=2_500_000, ls_rate=1.0, ls_iters=300),
    "batched_fp32": dict(grid=64, map_seed=102, n_ligands=256, lig_seed=203,
                         n_runs=10, pop_size=150, max_generations=10**6,
                         max_evals_per_run=2_500_000, ls_rate=0.06, ls_iters=300),
    "serving_fp16": dict(grid=96, map_seed=105, lig_seed=205,
                         n_runs=10, pop_size=150, max_generations=10**6,
                         max_evals_per_run=250_000, ls_rate=0.06, ls_iters=300),
    "paper_inputs": dict(grid=64, map_seed=102, lig_seed=206,
                         n_runs=10, pop_size=150, max_generations=10**6,
                         max_evals_per_run=2_500_000, ls_rate=0.06, ls_iters=300),
}

# the paper's three inputs: (atoms, rotatable bonds)
PAPER_INPUT_SIZES = {"small": (21, 2), "medium": (43, 15), "large": (108, 31)}
PAPER_NRUNS = (10, 100)

# search constants shared by every workload (ADADELTA and LGA operator rates)
SEARCH_DEFAULTS = dict(rho=0.8, eps=1e-2, crossover_rate=0.8, mutation_rate=0.02,
                       tournament_rate=0.6, elitism=1, mut_trans=2.0,
                       mut_rot=math.pi / 2, mut_tors=math.pi)


def type_params():
    return synth.make_type_params(TYPE_SEED)


def receptor(name: str) -> synth.Receptor:
    w = WORKLOADS[name]
    return synth.make_receptor(w["grid"], w["map_seed"])


def ligand(name: str) -> synth.Ligand:
    w = WORKLOADS[name]
    return synth.make_ligand(w["n_atoms"], w["n_torsions"], w["lig_seed"], type_params())


def paper_ligand(size: str) -> synth.Ligand:
    """Synthetic stand-in for one of the paper's three inputs ("small", "medium", "large")."""
    n, t = PAPER_INPUT_SIZES[size]
    k = list(PAPER_INPUT_SIZES).index(size)
    return synth.make_ligand(n, t, WORKLOADS["paper_inputs"]["lig_seed"] * 10 + k, type_params())


def batched_ligands(name: str = "batched_fp32", count: int | None = None):
    """Ligands of uniform size 10..100 atoms with 0..32 rotatable bonds (capped)."""
    w = WORKLOADS[name]
    n = w["n_ligands"] if count is None else count
    rng = np.random.default_rng([w["lig_seed"], 0xBA7C])
    out = []
    for i in range(n):
        na = int(rng.integers(10, 101))
        nt = int(rng.integers(0, 33))
        out.append(synth.make_ligand(na, nt, w["lig_seed"] * 100003 + i, type_params()))
    return out


def serving_sizes(count: int, seed: int = 205):
    """(n_atoms, n_torsions) for serving requests: LogNormal(ln 35, 0.5) atoms
    resampled into [10, 120], rotatable bonds = min(round(n/5), n-3, 32)."""
    rng = np.random.default_rng([seed, 0x5E77])
    out = []
    while len(out) < count:
        n = int(round(math.exp(rng.normal(math.log(35.0), 0.5))))
        if 10 <= n <= 120:
            out.append((n, min(int(round(n / 5)), n - 3, 32)))
    return out


def search_params(name: str, seed: int = 7, **over):
    w = WORKLOADS[name]
    p = dict(SEARCH_DEFAULTS)
    p.update(n_runs=w["n_runs"], pop_size=w["pop_size"], max_generations=w["max_generations"],
             max_evals_per_run=w["max_evals_per_run"], ls_rate=w["ls_rate"],
             ls_iters=w["ls_iters"], seed=seed)
    p.update(over)
    return p
