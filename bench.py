"""Benchmark of the docking hot path on one MI355X.

Default workload (batched_fp32): 256 synthetic ligands (10-100 atoms, 0-32 rotatable bonds)
docked together against one 64^3 FP32 map set, 10 LGA runs x 150 individuals each, 6 % local
search x 300 ADADELTA steps, through md_dock_batch (one launch per GA phase and size class for
every ligand, each generation a captured graph).  One step = one md_dock_batch call over the
whole batch: the initial populations and the first --generations generations (50 by default,
the cold, widely spread generations included); --full-budget runs each ligand's full
2.5M-evaluation budget (878 generations) instead.  Inputs (maps, ligands) are resident on the
device before the timed region.

Prints one JSON line.  value = energy+gradient evaluations per second (the ADADELTA steps, each
one energy and gradient evaluation) over the timed steps; ligands docked per second at the full
budget are derived from the total evaluation rate (labelled derived).  roofline: the
local-search kernel's algorithmic flops over its launch time, from one extra batch launched
phase by phase: each GA phase's launches (one per size class) run concurrently over the branch
streams, as in the timed graph, and HIP events on the dock's stream bracket the phase.  baselines: the plain single-ligand
FP32 path on the same GPU (md_dock of the 40-atom production ligand, 20 runs; and of 16 of the
batch's own ligands one after another).  cpu_baseline: the FP64 oracle's energy+gradient
evaluations per second on the host cores, on random poses of the batch's ligands (and of one
core alone).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--generations G] [--full-budget]
                    [--no-cpu-baseline]
                    [--workload batched_fp32|plain_fp32_production|serving_fp16|paper_inputs|eval_sweep]
                    [--ls adadelta|solis_wets]

--workload plain_fp32_production: one step = one complete md_dock of the 40-atom ligand
(20 runs x 150, 2.5M evaluations per run, local search on every individual); --ls solis_wets
runs it with the Solis-Wets local search and counts its energy-only evaluations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "plain_fp32_production"       # the single-ligand production dock
DEFAULT_WORKLOAD = "batched_fp32"
PEAK_FP32_VALU_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


PROFILES = {"adadelta": os.path.join(ROOT, "profiles", "k_local_search_plain_fp32_production.txt"),
            "solis_wets": os.path.join(ROOT, "profiles", "k_ga_solis_wets_plain_fp32_production.txt"),
            "batched": os.path.join(ROOT, "profiles", "k_ga_local_search_batched_fp32.txt"),
            "serving": os.path.join(ROOT, "profiles", "k_ga_local_search_serving_fp16.txt")}
KERNEL_SRC = os.path.join(ROOT, "paper_2203_02096_amd", "csrc", "kernels.hip")


def measured_profile(ls="adadelta"):
    """Figures from the committed rocprofv3 summary of the local-search kernel: HBM bytes per
    launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counts) and VALU issue utilisation
    (SQ_INSTS_VALU); None for each when the kernel source has changed since they were taken."""
    import hashlib
    none = {"traffic": None, "valu_issue_utilisation": None, "valu_instructions_per_eval": None,
            "l2_read_bytes_per_launch": None, "l2_hit_rate": None}
    try:
        text = open(PROFILES[ls]).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return none
    vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(" "))
    if vals.get("kernel_source_sha256", "").strip() != sha:
        return none
    traffic = next((vals[k] for k in ("traffic_bytes_per_launch", "traffic_bytes_per_generation",
                                      "traffic_bytes_per_request") if k in vals), "nan")
    out = {"traffic": float(traffic),
           "valu_issue_utilisation": float(vals["valu_issue_utilisation"]),
           "valu_instructions_per_eval": float(vals["valu_instructions_per_eval"])}
    for k in ("l2_read_bytes_per_launch", "l2_hit_rate"):
        out[k] = float(vals[k]) if k in vals else None
    return out


def flop_model(n_atoms, n_torsions, n_pairs, sum_moving):
    """Algorithmic flop-equivalents of one energy+gradient evaluation (transcendentals count 4):
    pose 24*sum_M + 21*N + 25*T + 30, grid 170*N, pairs 75*P, reductions 12*sum_M + 12*N + 10*T."""
    N, T, P, M = n_atoms, n_torsions, n_pairs, sum_moving
    return (24 * M + 21 * N + 25 * T + 30) + 170 * N + 75 * P + (12 * M + 12 * N + 10 * T)


def flop_model_energy(n_atoms, n_torsions, n_pairs, sum_moving):
    """Algorithmic flop-equivalents of one energy-only evaluation (a Solis-Wets trial point):
    pose 24*sum_M + 21*N + 25*T + 30, grid value 62*N, pair energies 53*P, energy sum N."""
    N, T, P, M = n_atoms, n_torsions, n_pairs, sum_moving
    return (24 * M + 21 * N + 25 * T + 30) + 62 * N + 53 * P + N


def bytes_model(n_atoms, map_bytes=4):
    """Algorithmic bytes of one evaluation: 8 corners x 3 maps per atom."""
    return 24 * map_bytes * n_atoms


def mix_roofline(md, dligs, ls_evals_each, seconds, map_bytes):
    """Roofline of a mix of ligands: the local searches' algorithmic flops (flop_model) and map
    bytes (bytes_model) summed over the ligands, over the wall time.  The bound is the VALU (as
    for the single ligand); the HBM fraction is stated beside it."""
    flops = byts = 0.0
    for d, n in zip(dligs, ls_evals_each):
        info = md.md_ligand_info(d)
        flops += n * flop_model(info["n_atoms"], info["n_torsions"], info["n_pairs"], info["sum_moving"])
        byts += n * bytes_model(info["n_atoms"], map_bytes)
    tf = flops / seconds / 1e12
    gbs = byts / seconds / 1e9
    return {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / PEAK_FP32_VALU_TFLOPS, "traffic": None,
            "frac_of_nonpacked_fp32": tf / (PEAK_FP32_VALU_TFLOPS / 2),
            "hbm_algorithmic_GBs": gbs, "hbm_peak_GBs": PEAK_HBM_GBS, "hbm_frac": gbs / PEAK_HBM_GBS,
            "scope": "whole job: every local-search evaluation over the wall time"}


def single_ligand_path(md, drec, dligs, params, sample):
    """The plain single-ligand path on the same GPU: md_dock of `sample` ligands (spread over the
    list) one after another with the same parameters.  Returns (local-search evals/s, ligands/s,
    indices)."""
    import torch
    idx = sorted(set(int(round(k)) for k in
                     [i * (len(dligs) - 1) / max(1, sample - 1) for i in range(sample)]))
    ls = 0
    md.md_dock(drec, dligs[idx[0]], params[idx[0]], want_xyz=False)       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in idx:
        P = params[k]
        gens = md.md_dock_planned_generations(P)
        n_ls = max(0, min(P.pop_size, math.ceil(P.ls_rate * P.pop_size - 1e-4)))
        md.md_dock(drec, dligs[k], P, want_xyz=False)
        ls += P.n_runs * gens * n_ls * P.ls_iters
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return ls / dt, len(idx) / dt, idx


# ------------------------------------------------------------------ CPU baseline (oracle)
def _oracle_worker(args):
    seed, budget_s, grad, workload = args
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"      # one thread per process: `cores` counts what is used
    import numpy as np
    from oracle import ligand as OL
    from oracle import scoring as S
    from workload import configs, synth
    rec = configs.receptor(workload)
    grid = S.make_grid(rec.maps, rec.origin, rec.spacing)
    if workload == "batched_fp32":
        # the batch's own ligands, every one in turn, so the sample has the batch's size mix
        ligs = configs.batched_ligands(workload)
        k0 = seed % len(ligs)
        ligs = ligs[k0:] + ligs[:k0]
    else:
        ligs = [configs.ligand(workload)]
    ols = [OL.from_synth(l) for l in ligs]
    genes = [synth.random_genes(l, rec, 64, seed=seed * 1000 + k, margin=2.0).astype(np.float64)
             for k, l in enumerate(ligs)]
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        k = n % len(ols)
        g = genes[k][(n // len(ols)) % 64]
        if grad:
            S.energy_and_gradient(grid, ols[k], g, want_margin=False)
        else:
            S.energy(grid, ols[k], g)
        n += 1
    return n, time.perf_counter() - t0


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(budget_s=10.0, grad=True, workload=WORKLOAD, one_core_s=0.0):
    """The FP64 oracle's evaluations per second: one process per host core (up to 16) for
    budget_s each, and, with one_core_s > 0, one process alone first."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    ctx = mp.get_context("spawn")
    one = None
    if one_core_s > 0:
        with ctx.Pool(1) as pool:
            n1, t1 = pool.map(_oracle_worker, [(999, one_core_s, grad, workload)])[0]
        one = n1 / t1
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(1000 + i, budget_s, grad, workload) for i in range(cores)])
    wall = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    per_proc = max(r[1] for r in res)
    what = ("the batch's 256 ligands in turn" if workload == "batched_fp32" else f"the {workload} ligand")
    out = {"value": n / per_proc, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle {'energy+gradient' if grad else 'energy'} of random poses of {what} "
                     f"on the 64^3 grid, one process per core, {budget_s:.0f} s each ({n} evals, "
                     f"{wall:.1f} s wall incl. start-up); CPU: {_cpu_name()}"}
    if one is not None:
        out["one_core_value"] = one
        out["one_core_sample"] = f"the same, one process alone for {one_core_s:.0f} s"
    return out


# ------------------------------------------------------------------ GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed region, one plain device copy of this size (a known-size "
                         "dispatch for calibrating byte counters under a profiler)")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=[WORKLOAD, "batched_fp32", "serving_fp16", "paper_inputs", "eval_sweep", "eval_phases"],
                    help="batched_fp32 (default): 256 ligands in one batch; plain_fp32_production: "
                         "one ligand, 20 runs; serving_fp16: Poisson arrivals into the server; "
                         "paper_inputs: the paper's three input sizes at 10 and 100 runs, docked "
                         "with each block size; eval_sweep: md_eval of 2^16..2^20 independent poses; "
                         "eval_phases: md_eval with and without gradient and torsions, then a search, for "
                         "per-phase instruction counts under a profiler")
    ap.add_argument("--generations", type=int, default=50,
                    help="batched_fp32: generations per step (the full budget takes 878)")
    ap.add_argument("--full-budget", action="store_true",
                    help="batched_fp32: each step docks every ligand to its full budget")
    ap.add_argument("--no-baselines", action="store_true",
                    help="batched_fp32, serving_fp16: leave out the single-ligand baselines (for profiler runs)")
    ap.add_argument("--rates", default="25,50,75,100,150",
                    help="serving_fp16: arrival rates (ligands/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serving_fp16: requests per rate")
    ap.add_argument("--ls", default="adadelta", choices=["adadelta", "solis_wets"],
                    help="local optimiser of the production dock (default adadelta, the headline; "
                         "solis_wets reports energy-only evaluations per second)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch plans (else every ligand size class is autotuned "
                         "on the receptor before the timed region)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the docking path has "
              f"no cross-GPU work to measure here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched_fp32":
        return bench_batched(args)
    if args.workload == "serving_fp16":
        return bench_serving(args)
    if args.workload == "paper_inputs":
        return bench_paper_inputs(args)
    if args.workload == "eval_sweep":
        return bench_eval_sweep(args)
    if args.workload == "eval_phases":
        return bench_eval_phases(args)

    # the oracle baseline runs first, in spawned processes, before this process touches the GPU
    base = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds, grad=args.ls != "solis_wets")

    import numpy as np
    import torch

    import paper_2203_02096_amd as md
    from workload import configs

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    md.lib()
    rec = configs.receptor(WORKLOAD)
    lig = configs.ligand(WORKLOAD)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    dlig = md.Ligand.from_synth(lig)
    info = md.md_ligand_info(dlig)
    sw = args.ls == "solis_wets"
    sp = configs.search_params(WORKLOAD, seed=args.seed, ls_method=args.ls)
    P = md.dock_params(**sp)
    gens = md.md_dock_planned_generations(P)
    n_ls = max(0, min(P.pop_size, math.ceil(sp["ls_rate"] * P.pop_size - 1e-4)))
    # tune the launch plan for this dock's local-search launches (n_runs x n_ls searches)
    tune = None if args.no_autotune else md.md_ligand_autotune(drec, dlig, n_starts=P.n_runs * n_ls)
    plan = md.md_ligand_get_plan(dlig)
    ls_evals = P.n_runs * gens * n_ls * P.ls_iters
    total_evals = P.n_runs * (P.pop_size + gens * ((P.pop_size - P.elitism) + n_ls * P.ls_iters))
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)
    torch.cuda.synchronize()
    md.md_profile_reset()
    md.md_profile_enable(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        res = md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)   # blocking
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    md.md_profile_enable(False)
    ls_ms, ls_n = md.md_profile_read("local_search")
    kern = {k: md.md_profile_read(k) for k in md.mdock.KERNELS}

    ms_per_step = 1e3 * elapsed / args.steps
    value = ls_evals / (elapsed / args.steps)
    evals_per_ls_launch = P.n_runs * n_ls * P.ls_iters
    fm = flop_model_energy if sw else flop_model
    flops_eval = fm(info["n_atoms"], info["n_torsions"], info["n_pairs"], info["sum_moving"])
    avg_ls_s = ls_ms / 1e3 / max(ls_n, 1)
    achieved_tflops = flops_eval * evals_per_ls_launch / avg_ls_s / 1e12
    hbm_gbs = bytes_model(info["n_atoms"]) * evals_per_ls_launch / avg_ls_s / 1e9
    lat_ms = np.array(lat) * 1e3
    prof = measured_profile(args.ls)
    out = {
        "metric": "energy evals/s (Solis-Wets)" if sw else "energy+gradient evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": "64^3 x 9 maps FP32, 0.375 A",
                   "n_atoms": info["n_atoms"], "n_torsions": info["n_torsions"],
                   "n_pairs": info["n_pairs"], "n_runs": P.n_runs, "pop_size": P.pop_size,
                   "max_evals_per_run": P.max_evals_per_run, "generations": gens,
                   "ls_rate": sp["ls_rate"], "ls_iters": P.ls_iters, "local_search": args.ls},
        "launch_plan": {**plan, "autotuned": tune is not None},
        "ligands_per_s": 1.0 / (elapsed / args.steps),
        "total_evals_per_s": total_evals / (elapsed / args.steps),
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_VALU_TFLOPS,
                     "traffic": prof["traffic"], "kernel": "k_ga_solis_wets" if sw else "k_ga_local_search",
                     "frac_of_nonpacked_fp32": achieved_tflops / (PEAK_FP32_VALU_TFLOPS / 2),
                     "valu_issue_utilisation": prof["valu_issue_utilisation"],
                     "valu_instructions_per_eval": prof["valu_instructions_per_eval"],
                     "flop_per_eval": flops_eval, "evals_per_launch": evals_per_ls_launch,
                     "avg_launch_ms": avg_ls_s * 1e3, "launches": ls_n,
                     "hbm_algorithmic_GBs": hbm_gbs, "hbm_frac": hbm_gbs / PEAK_HBM_GBS,
                     "l2_read_GBs": (prof["l2_read_bytes_per_launch"] / avg_ls_s / 1e9
                                     if prof["l2_read_bytes_per_launch"] else None),
                     "l2_hit_rate": prof["l2_hit_rate"]},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kern.items()},
        "best_energy": float(res["best_energy"][0]),
        "cpu_baseline": base,
    }
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def _common(md):
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    md.lib()


def bench_eval_phases(args):
    """Per-phase instruction budget of one evaluation: md_eval of 2^16 random poses of the
    production ligand with and without the gradient, and of the same atoms with no rotatable bond
    (no torsions, hence no intramolecular pairs), then md_local_search (300 ADADELTA steps) from
    the same starts; the default plan throughout.  Launched in that order, each `--warmup` +
    `--steps` times, so a profiler's per-dispatch counters (SQ_INSTS_VALU, ...) divided by the
    evaluations of each launch give the budget: the differences separate the gradient, the
    torsions and pairs, and the search step's own work."""
    import numpy as np
    import torch

    import paper_2203_02096_amd as md
    from workload import configs, synth
    _common(md)
    rec = configs.receptor(WORKLOAD)
    lig = configs.ligand(WORKLOAD)
    rigid = synth.Ligand(lig.xyz, lig.types, lig.charges, lig.bonds, np.zeros(0, np.int32), lig.root,
                         lig.type_params)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    n = 1 << 16
    stream = torch.cuda.current_stream()
    rows = []
    for name, L, grad, search in (("torsions8_gradient", lig, True, False), ("torsions8_energy", lig, False, False),
                                  ("rigid_gradient", rigid, True, False), ("rigid_energy", rigid, False, False),
                                  ("torsions8_search300", lig, True, True)):
        dlig = md.Ligand.from_synth(L)
        info = md.md_ligand_info(dlig)
        genes = torch.from_numpy(synth.random_genes(L, rec, n, seed=5, margin=2.0)).cuda()
        e = torch.empty(n, device="cuda")
        d = torch.empty(n, L.n_genes, device="cuda")
        out_g = torch.empty_like(genes)
        iters = 300 if search else 1

        def launch():
            if search:
                md.md_local_search(drec, dlig, genes, out_g, e, iters, stream=stream)
            else:
                md.md_eval(drec, dlig, genes, e, d if grad else None, stream=stream)
        for _ in range(args.warmup):
            launch()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            launch()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        rows.append({"variant": name, "evals_per_launch": n * iters, "ms_per_launch": ms,
                     "ns_per_eval": ms * 1e6 / (n * iters), "n_atoms": info["n_atoms"],
                     "n_torsions": info["n_torsions"], "n_pairs": info["n_pairs"],
                     "launches": args.warmup + args.steps})
        print(f"[eval_phases] {name}: {ms:.3f} ms per launch", file=sys.stderr, flush=True)
    out = {"metric": "energy+gradient evals/s (md_eval, independent poses)", "value": n / (rows[0]["ms_per_launch"] * 1e-3),
           "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": rows[0]["ms_per_launch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "eval_phases", "ligand": WORKLOAD, "poses": n}, "variants": rows}
    print(json.dumps(out), flush=True)


def bench_eval_sweep(args):
    """The evaluation alone (md_eval: energy and gradient of independent poses, no search) of the
    production ligand on its 64^3 FP32 maps, for 2^16 .. 2^20 random poses in the box; each size
    timed with HIP events over --steps launches after --warmup.  value = evaluations/s at 2^20."""
    import numpy as np
    import torch

    import paper_2203_02096_amd as md
    from workload import configs, synth
    _common(md)
    rec = configs.receptor(WORKLOAD)
    lig = configs.ligand(WORKLOAD)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    dlig = md.Ligand.from_synth(lig)
    info = md.md_ligand_info(dlig)
    tune = None if args.no_autotune else md.md_ligand_autotune(drec, dlig, n_starts=0)
    flops = flop_model(info["n_atoms"], info["n_torsions"], info["n_pairs"], info["sum_moving"])
    stream = torch.cuda.current_stream()
    rows = []
    for lg in range(16, 21):
        n = 1 << lg
        genes = torch.from_numpy(synth.random_genes(lig, rec, n, seed=lg, margin=2.0)).cuda()
        e = torch.empty(n, device="cuda")
        d = torch.empty(n, lig.n_genes, device="cuda")
        for _ in range(max(1, args.warmup)):
            md.md_eval(drec, dlig, genes, e, d, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            md.md_eval(drec, dlig, genes, e, d, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        rows.append({"poses": n, "ms_per_launch": ms, "evals_per_s": n / (ms * 1e-3),
                     "tflops": flops * n / (ms * 1e-3) / 1e12})
        print(f"[eval_sweep] {n} poses: {ms:.3f} ms, {n / (ms * 1e-3):.3e} evals/s", file=sys.stderr, flush=True)
    top = rows[-1]
    out = {"metric": "energy+gradient evals/s (md_eval, independent poses)", "value": top["evals_per_s"],
           "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": top["ms_per_launch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "eval_sweep", "ligand": WORKLOAD, "n_atoms": info["n_atoms"],
                      "n_torsions": info["n_torsions"], "n_pairs": info["n_pairs"]},
           "launch_plan": md.md_ligand_get_plan(dlig), "autotuned": tune is not None,
           "roofline": {"bound": "alu", "achieved": top["tflops"], "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": top["tflops"] / PEAK_FP32_VALU_TFLOPS, "traffic": None, "kernel": "k_eval",
                        "frac_of_nonpacked_fp32": top["tflops"] / (PEAK_FP32_VALU_TFLOPS / 2),
                        "hbm_algorithmic_GBs": bytes_model(info["n_atoms"]) * top["evals_per_s"] / 1e9,
                        "hbm_frac": bytes_model(info["n_atoms"]) * top["evals_per_s"] / 1e9 / PEAK_HBM_GBS},
           "sweep": rows}
    print(json.dumps(out), flush=True)


def bench_paper_inputs(args):
    """The paper's three inputs (synthetic ligands of 21, 43 and 108 atoms with 2, 15 and 31
    rotatable bonds) docked with 10 and 100 runs, once per block size -- 1, 2, 4 and 8 waves per
    block, i.e. 64 to 512 threads per workgroup, one pose per wave (the paper swept 32 to 256
    threads per workgroup for its large input; one pose per 64-lane wave rules out 32) -- once
    per pose size -- 2 and 4 waves sharing each local-search pose, i.e. 128 and 256 threads per
    pose, the counterpart of the paper's threads per individual -- and once with the autotuned
    plan.  Each case is the median of --steps docks after --warmup; value is the local-search
    evaluations per second summed over the six (input, runs) cases at the best plan of each."""
    import numpy as np
    import torch

    import paper_2203_02096_amd as md
    from workload import configs
    _common(md)
    name = "paper_inputs"
    rec = configs.receptor(name)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    stream = torch.cuda.current_stream()
    cases = []
    total_ls, total_s = 0, 0.0
    for size in configs.PAPER_INPUT_SIZES:
        lig = configs.paper_ligand(size)
        dlig = md.Ligand.from_synth(lig)
        info = md.md_ligand_info(dlig)
        default = md.md_ligand_get_plan(dlig)
        for nruns in configs.PAPER_NRUNS:
            sp = configs.search_params(name, seed=args.seed, n_runs=nruns, ls_method=args.ls)
            P = md.dock_params(**sp)
            gens = md.md_dock_planned_generations(P)
            n_ls = max(0, min(P.pop_size, math.ceil(sp["ls_rate"] * P.pop_size - 1e-4)))
            ls_evals = nruns * gens * n_ls * P.ls_iters

            def timed():
                for _ in range(args.warmup):
                    md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)
                ts = []
                for _ in range(args.steps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)
                    ts.append(time.perf_counter() - t0)
                print(f"[paper_inputs] {size} nruns {nruns} plan {md.md_ligand_get_plan(dlig)}: "
                      f"{float(np.median(ts)):.3f} s", file=sys.stderr, flush=True)
                return float(np.median(ts))

            per_wpb, per_wpp = {}, {}
            for wpb in (1, 2, 4, 8):
                try:
                    md.md_ligand_set_plan(dlig, default["lds_budget"], default["group_div"], wpb)
                except md.MdockError:
                    per_wpb[64 * wpb] = None        # the plan does not fit in LDS
                    continue
                per_wpb[64 * wpb] = timed()
            per_wpp[64] = per_wpb[64]
            for wpp in (2, 4):
                try:
                    md.md_ligand_set_plan(dlig, default["lds_budget"], default["group_div"], wpp, wpp)
                except md.MdockError:
                    per_wpp[64 * wpp] = None
                    continue
                per_wpp[64 * wpp] = timed()
            md.md_ligand_set_plan(dlig, default["lds_budget"], default["group_div"], default["waves_per_block"])
            tune = md.md_ligand_autotune(drec, dlig, n_starts=nruns * n_ls, force=True)
            t_tuned = timed()
            md.md_ligand_set_plan(dlig, default["lds_budget"], default["group_div"], default["waves_per_block"])
            ok = [t for t in per_wpb.values() if t is not None]
            best = min(ok + [t for t in per_wpp.values() if t is not None] + [t_tuned])
            total_ls += ls_evals
            total_s += best
            cases.append({"input": size, "n_atoms": info["n_atoms"], "n_torsions": info["n_torsions"],
                          "n_pairs": info["n_pairs"], "n_runs": nruns, "generations": gens,
                          "seconds_by_threads_per_block": per_wpb, "seconds_by_threads_per_pose": per_wpp,
                          "seconds_tuned": t_tuned,
                          "tuned_plan": tune["plan"], "worst_over_best": max(ok) / min(ok),
                          "ls_evals_per_s_best": ls_evals / best})
            print(f"[paper_inputs] {size} nruns {nruns}: threads per block " +
                  ", ".join(f"{k}: {v:.3f} s" if v is not None else f"{k}: n/a" for k, v in per_wpb.items()) +
                  "; threads per pose " +
                  ", ".join(f"{k}: {v:.3f} s" if v is not None else f"{k}: n/a" for k, v in per_wpp.items()) +
                  f"; tuned {t_tuned:.3f} s {tune['plan']}", file=sys.stderr, flush=True)
    out = {
        "metric": ("energy evals/s (Solis-Wets)" if args.ls == "solis_wets" else "energy+gradient evals/s"),
        "value": total_ls / total_s,
        "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * total_s, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "grid": "64^3 x 9 maps FP32", "pop_size": 150,
                   "max_evals_per_run": 2_500_000, "ls_rate": 0.06, "ls_iters": 300,
                   "local_search": args.ls},
        "cases": cases,
    }
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """256 ligands (10-100 atoms, 0-32 rotatable bonds) against one 64^3 FP32 map set, 10 runs x
    150 each, docked together through md_dock_batch (one launch per GA phase and size class for
    all of them).  One step = one md_dock_batch call: initial populations and --generations
    generations (--full-budget: each ligand's whole budget).  value = ADADELTA evaluations per
    second over the timed steps; ligands/s at the full 2.5M-evaluation budget are derived from the
    total evaluation rate."""
    name = "batched_fp32"
    # the oracle baseline runs first, in spawned processes, before this process touches the GPU
    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(args.cpu_seconds, workload=name, one_core_s=min(args.cpu_seconds, 8.0))
    import numpy as np
    import torch

    import paper_2203_02096_amd as md
    from workload import configs
    _common(md)
    rec = configs.receptor(name)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    ligs = configs.batched_ligands(name)
    dligs = [md.Ligand.from_synth(l) for l in ligs]
    infos = [md.md_ligand_info(d) for d in dligs]
    full = md.dock_params(**configs.search_params(name, seed=args.seed))
    full_gens = md.md_dock_planned_generations(full)
    gens = full_gens if args.full_budget else max(1, min(args.generations, full_gens))
    sp = configs.search_params(name, seed=args.seed, max_generations=gens)
    P = md.dock_params(**sp)
    jobs = [(d, P) for d in dligs]
    # plan policy chosen by timing the candidate policies on this batch (untimed setup)
    t_tune = time.perf_counter()
    tuned = None if args.no_autotune else md.md_batch_autotune(drec, jobs, generations=9)
    t_tune = time.perf_counter() - t_tune
    plan_mix = {}
    for dl in dligs:
        pl = md.md_ligand_get_plan(dl)
        key = (f"{'A2' if dl.n_atoms > 64 else 'A1'}_wpb{pl['waves_per_block']}_wpp{pl['waves_per_pose']}"
               f"_lds{pl['lds_budget'] // 1024}k")
        plan_mix[key] = plan_mix.get(key, 0) + 1
    n_ls = max(0, min(P.pop_size, math.ceil(sp["ls_rate"] * P.pop_size - 1e-4)))
    per_gen = (P.pop_size - P.elitism) + n_ls * P.ls_iters
    total_evals = len(jobs) * P.n_runs * (P.pop_size + gens * per_gen)
    ls_evals = len(jobs) * P.n_runs * gens * n_ls * P.ls_iters
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        md.md_dock_batch(drec, jobs, stream=stream, want_xyz=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        res = md.md_dock_batch(drec, jobs, stream=stream, want_xyz=False)   # blocking
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # one more step launched phase by phase with HIP events (md_profile_*) for the roofline
    md.md_profile_reset()
    md.md_profile_enable(True)
    md.md_dock_batch(drec, jobs, stream=stream, want_xyz=False)
    torch.cuda.synchronize()
    md.md_profile_enable(False)
    kern = {k: md.md_profile_read(k) for k in md.mdock.KERNELS}
    ls_ms, ls_n = kern["local_search"]
    ls_each = P.n_runs * gens * n_ls * P.ls_iters
    flops = sum(ls_each * flop_model(i["n_atoms"], i["n_torsions"], i["n_pairs"], i["sum_moving"]) for i in infos)
    byts = sum(ls_each * bytes_model(i["n_atoms"]) for i in infos)
    ls_s = ls_ms / 1e3
    tf = flops / ls_s / 1e12
    prof = measured_profile("batched")
    sizes = np.array([l.n_atoms for l in ligs])
    evals_per_ligand_full = P.n_runs * (P.pop_size + full_gens * per_gen)
    rate = total_evals / dt
    lat_ms = np.array(lat) * 1e3

    # a known-size plain copy after the profiled step (calibrates byte counters under a profiler)
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    # the plain single-ligand FP32 path on the same GPU: the 40-atom production dock, and 16 of
    # the batch's own ligands docked one after another with the batch's parameters
    prod = None
    single_eps = single_lps = single_flops = single_ls = None
    idx = []
    if not args.no_baselines:
        prod = single_ligand_production(md, args)
        single_eps, single_lps, idx = single_ligand_path(md, drec, dligs, [P] * len(dligs), 16)
        single_flops = sum(P.n_runs * gens * n_ls * P.ls_iters *
                           flop_model(infos[k]["n_atoms"], infos[k]["n_torsions"], infos[k]["n_pairs"],
                                      infos[k]["sum_moving"]) for k in idx)
        single_ls = len(idx) * P.n_runs * gens * n_ls * P.ls_iters
    out = {"metric": "energy+gradient evals/s", "value": ls_evals / dt, "unit": "evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": name, "grid": "64^3 x 9 maps FP32, 0.375 A", "n_ligands": len(ligs),
                      "atoms": [int(sizes.min()), int(sizes.max())], "mean_atoms": float(sizes.mean()),
                      "n_runs": P.n_runs, "pop_size": P.pop_size, "generations_per_step": gens,
                      "full_budget_generations": full_gens, "ls_rate": sp["ls_rate"], "ls_iters": P.ls_iters,
                      "max_evals_per_run": full.max_evals_per_run},
           "total_evals_per_s": rate,
           "ligands_per_s": (len(jobs) / dt) if gens == full_gens else rate / evals_per_ligand_full,
           "ligands_per_s_kind": ("measured: every ligand docked to its full budget in each step"
                                  if gens == full_gens else
                                  f"derived: total evals/s / {evals_per_ligand_full} evals per ligand at the "
                                  f"full budget ({full_gens} generations)"),
           "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                          "what": "per step (the whole batch)"},
           "autotune": {**(tuned or {"policy": "default (not tuned)"}), "seconds": t_tune, "plan_mix": plan_mix},
           "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / PEAK_FP32_VALU_TFLOPS, "traffic": prof["traffic"],
                        "traffic_unit": "HBM bytes per generation of local-search launches",
                        "kernel": "k_ga_local_search (every size class)",
                        "frac_of_nonpacked_fp32": tf / (PEAK_FP32_VALU_TFLOPS / 2),
                        "valu_issue_utilisation": prof["valu_issue_utilisation"],
                        "valu_instructions_per_eval": prof["valu_instructions_per_eval"],
                        "flop_per_generation": flops / gens, "algorithmic_bytes_per_generation": byts / gens,
                        "ls_ms_per_generation": ls_ms / gens, "ls_phases": ls_n,
                        "hbm_algorithmic_GBs": byts / ls_s / 1e9, "hbm_frac": byts / ls_s / 1e9 / PEAK_HBM_GBS,
                        "l2_read_GBs": (prof["l2_read_bytes_per_launch"] / (ls_s / gens) / 1e9
                                        if prof["l2_read_bytes_per_launch"] else None),
                        "l2_hit_rate": prof["l2_hit_rate"],
                        "scope": "one extra step launched phase by phase (each phase's size-class launches "
                                 "concurrent, as in the timed graph; HIP events on the dock's stream bracket "
                                 "the phase): algorithmic flops of the local-search phases over their summed "
                                 "time"},
           "whole_job_tflops": flops / dt / 1e12,
           "baselines": None if args.no_baselines else {
               "single_ligand_production": prod,
               "batch_ligands_alone": {"evals_per_s": single_eps, "ligands": len(idx),
                                       "tflops": single_flops / (single_ls / single_eps) / 1e12,
                                       "speedup_of_batch": (ls_evals / dt) / single_eps,
                                       "what": "md_dock of 16 of the batch's ligands one after another, same "
                                               "parameters and plans, same GPU"}},
           "kernel_ms_per_step": {k: v[0] for k, v in kern.items()},
           "kernel_ms_note": "the extra step launched phase by phase (HIP events around each phase's "
                             "concurrent size-class launches); the timed steps replay each generation as a "
                             "HIP graph",
           "best_energy_job0": float(res[0]["best_energy"][0]),
           "cpu_baseline": base}
    print(json.dumps(out), flush=True)


def single_ligand_production(md, args, docks=3):
    """The plain single-ligand FP32 path: md_dock of the 40-atom production ligand (20 runs x 150,
    2.5M evaluations per run, local search on every individual), default plan."""
    import torch
    from workload import configs
    rec = configs.receptor(WORKLOAD)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp32")
    dlig = md.Ligand.from_synth(configs.ligand(WORKLOAD))
    info = md.md_ligand_info(dlig)
    sp = configs.search_params(WORKLOAD, seed=args.seed)
    P = md.dock_params(**sp)
    gens = md.md_dock_planned_generations(P)
    n_ls = max(0, min(P.pop_size, math.ceil(sp["ls_rate"] * P.pop_size - 1e-4)))
    ls = P.n_runs * gens * n_ls * P.ls_iters
    stream = torch.cuda.current_stream()
    md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(docks):
        md.md_dock(drec, dlig, P, stream=stream, want_xyz=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / docks
    fl = flop_model(info["n_atoms"], info["n_torsions"], info["n_pairs"], info["sum_moving"])
    return {"evals_per_s": ls / dt, "ligands_per_s": 1.0 / dt, "ms_per_dock": dt * 1e3,
            "tflops": ls * fl / dt / 1e12, "docks": docks,
            "what": "md_dock of the 40-atom / 8-torsion ligand on its 64^3 FP32 maps, 20 runs x 150, "
                    "2.5M evaluations per run, local search on every individual (whole dock, default plan)"}


def bench_serving(args):
    """Requests arrive as a Poisson stream at each rate; every request is 10 runs x 150 with a
    250k-evaluation budget per run against a 96^3 map set stored in FP16, for a ligand of
    log-normal size (median 35 atoms, 10-120).  The server batches resident requests
    continuously; latency = completion - arrival."""
    import numpy as np

    import paper_2203_02096_amd as md
    from workload import configs, synth
    _common(md)
    name = "serving_fp16"
    rec = configs.receptor(name)
    drec = md.Receptor(rec.maps, rec.origin, rec.spacing, "fp16")
    sizes = configs.serving_sizes(args.requests, seed=205)
    ligs = [md.Ligand.from_synth(synth.make_ligand(n, t, 9000 + k, configs.type_params()))
            for k, (n, t) in enumerate(sizes)]
    sp = configs.search_params(name, seed=args.seed)
    # plan policy timed on a batch of request ligands (untimed setup), applied to all of them
    t_tune = time.perf_counter()
    tuned = None
    if not args.no_autotune:
        tuned = md.md_batch_autotune(drec, [(l, md.dock_params(**sp)) for l in ligs[:96]], generations=9)
        if tuned["policy"] != "default":
            pol = {"tuned_alone": None, "lds_all": dict(lds_budget=160 * 1024), "wide_blocks": dict(waves_per_block=8),
                   "small_groups": dict(group_div=2),
                   "shared_large": dict(waves_per_block=4, waves_per_pose=4),
                   "full_blocks": dict(waves_per_block=16, lds_budget=160 * 1024)}[tuned["policy"]]
            for l in ligs[96:]:
                if pol is None:
                    md.md_ligand_autotune(drec, l)
                elif tuned["policy"] != "shared_large" or l.n_atoms > 64:
                    md.md_ligand_set_plan(l, **{"lds_budget": 65536, "group_div": 3, "waves_per_block": 4, **pol})
    t_tune = time.perf_counter() - t_tune
    plan_mix = {}
    for l in ligs:
        pl = md.md_ligand_get_plan(l)
        key = f"wpb{pl['waves_per_block']}_wpp{pl['waves_per_pose']}_lds{pl['lds_budget'] // 1024}k"
        plan_mix[key] = plan_mix.get(key, 0) + 1
    P = md.dock_params(**sp)
    n_ls = max(0, min(P.pop_size, math.ceil(sp["ls_rate"] * P.pop_size - 1e-4)))
    gens = md.md_dock_planned_generations(P)
    evals_per_req = P.n_runs * (P.pop_size + gens * ((P.pop_size - P.elitism) + n_ls * P.ls_iters))
    # a known-size plain copy before the served requests: calibrates byte counters under a
    # profiler and marks where the requests' dispatches begin (the plan tuning's end before it)
    if args.copy_mib > 0:
        import torch
        src = torch.ones(args.copy_mib * (1 << 20) // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        srv = md.Server(drec, hbm_budget_bytes=8 << 30, max_slots=256)
        rng = np.random.default_rng([args.seed, int(rate)])
        gaps = rng.exponential(1.0 / rate, len(ligs))
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        for k, lig in enumerate(ligs):
            t_next += gaps[k]
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            p = md.dock_params(**{**sp, "seed": args.seed * 1000 + k})
            tickets.append(srv.submit(lig, p))
            if k % 500 == 499:
                print(f"[serving] rate {rate:g}/s: {k + 1} submitted", file=sys.stderr, flush=True)
        for t in tickets:
            srv.wait(t, want_xyz=False)
        t_end = time.perf_counter()
        times = np.array([srv.times(t) for t in tickets])     # submit, start, end (monotonic host clock)
        lat = (times[:, 2] - times[:, 0]) * 1e3
        st = srv.stats()
        srv.close()
        # steady window: requests that arrived after the first 10 % and before the last 10 % of
        # the arrivals (the warm-up and the drain left out); throughput over the same window
        n = len(tickets)
        lo, hi = n // 10, n - n // 10
        steady = lat[lo:hi]
        win = times[hi - 1, 0] - times[lo, 0]
        done_in = np.sum((times[:, 2] >= times[lo, 0]) & (times[:, 2] <= times[hi - 1, 0]))
        results.append({"rate": rate, "requests": n, "p50_ms": float(np.percentile(steady, 50)),
                        "p99_ms": float(np.percentile(steady, 99)),
                        "ligands_per_s": float(done_in / win) if win > 0 else None,
                        "ligands_per_s_whole": n / (times[:, 2].max() - times[:, 0].min()),
                        "offered_per_s": float((hi - 1 - lo) / win) if win > 0 else None,
                        "evals_per_s": float(done_in / win) * evals_per_req if win > 0 else None,
                        "wall_s": t_end - t_start, "span_s": float(times[:, 2].max() - times[:, 0].min()),
                        "ticks": st["ticks"], "busy_s": st["busy_seconds"]})
        print(json.dumps({"partial": results[-1]}), file=sys.stderr, flush=True)
    # capacity: the completion rate once the offered rate exceeds it (the largest steady
    # completion rate measured)
    capacity = max(r["ligands_per_s"] or 0.0 for r in results)
    best = max(results, key=lambda r: r["ligands_per_s"] or 0.0)
    ls_per_req = P.n_runs * gens * n_ls * P.ls_iters
    roof = mix_roofline(md, ligs, [ls_per_req] * len(ligs), best["span_s"], 2)
    prof = measured_profile("serving")
    roof.update({"traffic": prof["traffic"], "traffic_unit": "HBM bytes per request of local-search launches",
                 "valu_issue_utilisation": prof["valu_issue_utilisation"],
                 "valu_instructions_per_eval": prof["valu_instructions_per_eval"], "l2_hit_rate": prof["l2_hit_rate"]})
    single_eps = single_lps = None
    idx = []
    if not args.no_baselines:
        single_eps, single_lps, idx = single_ligand_path(
            md, drec, ligs, [md.dock_params(**{**sp, "seed": args.seed * 1000 + k}) for k in range(len(ligs))], 16)
    out = {"metric": "ligands docked/s (serving)", "value": capacity, "unit": "ligands/s",
           "n_gpus": 1, "steps": len(results), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": name, "grid": "96^3 x 9 maps FP16", "requests_per_rate": len(ligs),
                      "n_runs": P.n_runs, "pop_size": P.pop_size, "generations": gens,
                      "evals_per_request": evals_per_req, "median_atoms": float(np.median([n for n, _ in sizes]))},
           "autotune": {**(tuned or {"policy": "default (not tuned)"}), "seconds": t_tune, "plan_mix": plan_mix},
           "roofline": {**roof, "scope": f"the {best['rate']:g}/s run: every local-search evaluation over the "
                                          f"span from the first arrival to the last completion"},
           "ls_evals_per_s": len(ligs) * ls_per_req / best["span_s"],
           "single_ligand_path": {"ligands_per_s": single_lps, "evals_per_s": single_eps,
                                  "speedup_of_serving": best["ligands_per_s"] / single_lps if single_lps else None,
                                  "ligands": len(idx),
                                  "what": "md_dock of 16 of the requests one after another, same parameters "
                                          "and plans, same GPU"},
           "capacity_ligands_per_s": capacity,
           "capacity_note": "the largest steady-window completion rate over the offered rates; rates below it "
                            "are served as they arrive (latency = one dock plus queueing), rates above it "
                            "queue up",
           "rates": results}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
