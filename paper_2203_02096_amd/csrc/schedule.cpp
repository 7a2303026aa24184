// Per-generation launch schedule of the job-table GA kernels, shared by md_dock_batch and the
// docking server, and its capture as a HIP graph.
//
// Ligands of very different sizes go through the same generation (the paper's screening
// workflow docks a heterogeneous ligand stream; its discussion of heterogeneously sized
// ligands makes load balance part of the problem).  Two choices here keep one large ligand
// from setting the cost of many small ones:
//  * size classes: jobs are grouped by atoms per lane and by how many blocks of their LDS
//    plan fit on a compute unit, and each group is one launch with that group's LDS size, so
//    a small ligand never runs with a large ligand's LDS reservation (and lower occupancy);
//  * longest first: inside a launch, the blocks of the most expensive jobs come first, so the
//    long waves start early and the short ones fill the tail.
// One generation (selection/crossover/mutation + evaluation, local-search picks, local search,
// epilogue) reads everything it needs from the device job table, so the same sequence of
// launches serves every generation and is captured once and replayed.
#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>

#include "internal.h"
#include "mdock.h"

namespace mdock {

namespace {

constexpr int kLdsPerCu = 160 * 1024;
constexpr size_t kGraphBranches = 4;   // concurrent size-class launches in a captured phase

// blocks of this LDS size that fit on one compute unit
int occupancy_class(int lds) { return lds <= 0 ? 64 : std::min(64, kLdsPerCu / lds); }

// Relative cost of one evaluation (pair slots dominate; atoms and torsions add the rest).
double eval_cost(const LigDev& L) {
  return (double)L.n_rows * kWave + 8.0 * L.n_atoms + 16.0 * L.n_tors + 64.0;
}

}  // namespace

void build_schedule(const std::vector<SchedJob>& jobs, GenSchedule& out) {
  out = GenSchedule();
  // bucket key: (atoms per lane, waves per block, occupancy class); larger classes first
  using Key = std::tuple<int, int, int>;
  std::map<Key, std::vector<int>> pop_b, ls_b;
  for (int k = 0; k < (int)jobs.size(); ++k) {
    const SchedJob& j = jobs[k];
    const int A = j.L->n_atoms > kWave ? 2 : 1;
    const Key key(A, j.L->wpb, -occupancy_class(j.L->lds_bytes) * j.L->wpb);
    pop_b[key].push_back(k);
    if (j.n_ls > 0) ls_b[key].push_back(k);
  }
  auto emit = [&](std::map<Key, std::vector<int>>& buckets, bool ls, std::vector<PhaseLaunch>& launches) {
    for (auto& kv : buckets) {
      std::vector<int>& members = kv.second;
      std::vector<double> cost(jobs.size(), 0.0);
      for (int k : members) {
        const SchedJob& j = jobs[k];
        cost[k] = eval_cost(*j.L) * (ls ? (double)j.ls_iters : 1.0);
      }
      std::stable_sort(members.begin(), members.end(), [&](int a, int b) { return cost[a] > cost[b]; });
      PhaseLaunch pl;
      pl.A = std::get<0>(kv.first);
      pl.wpb = std::get<1>(kv.first);
      pl.lds = 0;
      pl.first = (int)out.blocks.size();
      for (int k : members) {
        const SchedJob& j = jobs[k];
        const long long waves = ls ? (long long)j.n_runs * j.n_ls : (long long)j.n_runs * j.pop_size;
        for (long long w = 0; w < waves; w += pl.wpb) out.blocks.push_back(make_int2(j.slot, (int)w));
        pl.lds = std::max(pl.lds, j.L->lds_bytes);
      }
      pl.count = (int)out.blocks.size() - pl.first;
      if (pl.count > 0) launches.push_back(pl);
    }
  };
  emit(pop_b, false, out.pop);
  emit(ls_b, true, out.ls);
  out.run_first = (int)out.blocks.size();
  for (const SchedJob& j : jobs)
    if (j.n_ls > 0)
      for (int r = 0; r < j.n_runs; r += kWavesPerBlock) out.blocks.push_back(make_int2(j.slot, r));
  out.run_count = (int)out.blocks.size() - out.run_first;
}

hipError_t launch_init_phase(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                             hipStream_t s, const LaunchHook* hook) {
  hipError_t e = hipSuccess;
  for (const PhaseLaunch& pl : g.pop) {
    auto f = [&] { return launch_ga_init(table, d_blocks + pl.first, pl.count, pl.A, pl.wpb, pl.lds, R, s); };
    e = hook ? (*hook)(MD_K_INIT_POPULATION, f) : f();
    if (e != hipSuccess) return e;
  }
  return e;
}

namespace {

// Launches the phase's size-class launches one after another on s, or, with side streams,
// forked across s and the side streams (joined back into s before returning): during graph
// capture that makes them parallel branches, so one class's tail overlaps another's work.
hipError_t launch_phase(const std::vector<PhaseLaunch>& launches, hipStream_t s,
                        const std::vector<hipStream_t>* side, int kind, const LaunchHook* hook,
                        const std::function<hipError_t(const PhaseLaunch&, hipStream_t)>& one) {
  hipError_t e = hipSuccess;
  if (!side || side->empty() || launches.size() < 2) {
    for (const PhaseLaunch& pl : launches) {
      auto f = [&] { return one(pl, s); };
      e = hook ? (*hook)(kind, f) : f();
      if (e != hipSuccess) return e;
    }
    return e;
  }
  const size_t n_side = std::min(side->size(), launches.size() - 1);
  std::vector<hipEvent_t> ev(1 + n_side, nullptr);
  for (hipEvent_t& x : ev) {
    e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  for (size_t k = 0; k < n_side && e == hipSuccess; ++k) e = hipStreamWaitEvent((*side)[k], ev[0], 0);
  for (size_t i = 0; i < launches.size() && e == hipSuccess; ++i)
    e = one(launches[i], i == 0 ? s : (*side)[(i - 1) % n_side]);
  for (size_t k = 0; k < n_side && e == hipSuccess; ++k) e = hipEventRecord(ev[1 + k], (*side)[k]);
  for (size_t k = 0; k < n_side && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, ev[1 + k], 0);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  return e;
}

}  // namespace

hipError_t launch_generation_phase(const GenSchedule& g, JobDev* table, int n_table, const int2* d_blocks,
                                   const RecDev& R, hipStream_t s, const LaunchHook* hook,
                                   const std::vector<hipStream_t>* side) {
  hipError_t e = launch_phase(g.pop, s, side, MD_K_GENERATION, hook, [&](const PhaseLaunch& pl, hipStream_t st) {
    return launch_ga_generation(table, d_blocks + pl.first, pl.count, pl.A, pl.wpb, pl.lds, R, st);
  });
  if (e != hipSuccess) return e;
  auto run = [&](int kind, const std::function<hipError_t()>& f) { return hook ? (*hook)(kind, f) : f(); };
  if (g.run_count > 0) {
    e = run(MD_K_LS_PICK, [&] { return launch_ga_ls_pick(table, d_blocks + g.run_first, g.run_count, s); });
    if (e != hipSuccess) return e;
  }
  e = launch_phase(g.ls, s, side, MD_K_LOCAL_SEARCH, hook, [&](const PhaseLaunch& pl, hipStream_t st) {
    return launch_ga_local_search(table, d_blocks + pl.first, pl.count, pl.A, pl.wpb, pl.lds, R, st);
  });
  if (e != hipSuccess) return e;
  return run(MD_K_SUM_EVALS, [&] { return launch_ga_advance(table, n_table, s); });
}

// ------------------------------------------------------------------ captured generation
hipError_t GenGraph::capture(const GenSchedule& g, JobDev* table, int n_table, const int2* d_blocks,
                             const RecDev& R) {
  reset();
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  // side streams for the parallel branches of the phases with several size-class launches
  std::vector<hipStream_t> side;
  size_t width = 1;
  for (const auto* v : {&g.pop, &g.ls}) width = std::max(width, v->size());
  for (size_t k = 0; k + 1 < std::min<size_t>(width, kGraphBranches) && e == hipSuccess; ++k) {
    hipStream_t x = nullptr;
    e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (e == hipSuccess) side.push_back(x);
  }
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t el = launch_generation_phase(g, table, n_table, d_blocks, R, cs, nullptr, &side);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess && exec_) {
      (void)hipGraphExecDestroy(exec_);
      exec_ = nullptr;
    }
  }
  for (hipStream_t x : side) (void)hipStreamDestroy(x);
  (void)hipStreamDestroy(cs);
  return e;
}

hipError_t GenGraph::launch(hipStream_t s) const {
  return exec_ ? hipGraphLaunch(exec_, s) : hipErrorInvalidValue;
}

void GenGraph::reset() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  exec_ = nullptr;
}

namespace {
bool g_use_graphs = true;
}

bool use_graphs() { return g_use_graphs; }
void set_use_graphs(bool on) { g_use_graphs = on; }

}  // namespace mdock
