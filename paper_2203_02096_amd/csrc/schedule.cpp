// Per-generation launch schedule of the job-table GA kernels, shared by md_dock_batch and the
// docking server, and its capture as a HIP graph.
//
// Ligands of very different sizes go through the same launches (the paper's screening
// workflow docks a heterogeneous ligand stream; its discussion of heterogeneously sized
// ligands makes load balance part of the problem).  Three choices here keep large ligands from
// setting the pace of small ones:
//  * size classes: jobs are grouped by atoms per lane, waves per block and how many blocks of
//    their LDS plan fit on a compute unit; each class has its own chain of launches with the
//    class's LDS size, so a small ligand never runs with a large ligand's LDS reservation --
//    except that a class too small to fill the device joins a larger class whose reservation
//    covers it, rather than run alone as a latency-bound tail;
//  * longest first: inside a launch, the blocks of the most expensive jobs come first, so the
//    long waves start early and the short ones fill the tail;
//  * independent chains: a class's generation (selection/crossover/mutation + evaluation,
//    local-search picks, local search, epilogue) depends only on its own jobs, so in a captured
//    phase the classes are parallel graph branches, and a cheap class may run several
//    generations while an expensive one runs one.
// Every kernel reads what it needs from the device job table (a finished job's work is skipped
// on the device), so the same captured phase serves every generation and is replayed.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>

#include "internal.h"
#include "mdock.h"

namespace mdock {

namespace {

constexpr int kLdsPerCu = 160 * 1024;
constexpr size_t kGraphBranches = 4;   // streams for the classes' parallel branches

// a Solis-Wets evaluation (energy only) relative to an ADADELTA step (energy and gradient)
constexpr double kEnergyOnlyCost = 0.7;   // measured: 1.98 vs 2.82 ms per production launch

// blocks of this LDS size that fit on one compute unit
int occupancy_class(int lds) { return lds <= 0 ? 64 : std::min(64, kLdsPerCu / lds); }

// Relative cost of one evaluation (pair slots dominate; atoms and torsions add the rest).
double eval_cost(const LigDev& L) {
  return (double)L.n_rows * kWave + 8.0 * L.n_atoms + 16.0 * L.n_tors + 64.0;
}

}  // namespace

void build_schedule(const std::vector<SchedJob>& jobs, GenSchedule& out, int max_reps, int uniform_reps) {
  out = GenSchedule();
  // class key: (atoms per lane, waves per block, -(waves per CU), local optimiser, waves per
  // search); denser classes first
  using Key = std::tuple<int, int, int, int, int>;
  std::map<Key, std::vector<int>> cls;
  for (int k = 0; k < (int)jobs.size(); ++k) {
    const SchedJob& j = jobs[k];
    const int A = j.L->n_atoms > kWave ? 2 : 1;
    cls[Key(A, j.L->wpb, -occupancy_class(j.L->lds_bytes) * j.L->wpb, j.ls_method, std::max(1, j.L->wpp))]
        .push_back(k);
  }
  // A class too small to fill the device on its own (fewer local-search waves than a quarter of
  // the device's wave slots) runs as a tail of its own launches, one search's latency long,
  // whichever its ligands' plans.  Such a class joins the largest class of the same atoms per
  // lane, waves per block, local optimiser and waves per search whose LDS reservation already
  // covers its plans (its blocks then take that reservation): its searches, longest first, then
  // fill the larger launch's tail.  Plans, and so results, are unchanged.
  {
    constexpr long long kSmallClassWaves = 1024;
    std::map<Key, long long> waves;
    std::map<Key, int> lds;
    for (const auto& kv : cls)
      for (int k : kv.second) {
        const SchedJob& j = jobs[k];
        waves[kv.first] += (long long)j.n_runs * j.n_ls * std::max(1, j.L->wpp);
        lds[kv.first] = std::max(lds[kv.first], j.L->lds_bytes);
      }
    std::vector<Key> order;
    for (const auto& kv : cls) order.push_back(kv.first);
    std::stable_sort(order.begin(), order.end(), [&](const Key& a, const Key& b) { return waves[a] < waves[b]; });
    for (const Key& small : order) {
      if (waves[small] >= kSmallClassWaves || !cls.count(small)) continue;
      const Key* into = nullptr;
      for (const auto& kv : cls) {
        const Key& k = kv.first;
        if (k == small || std::get<0>(k) != std::get<0>(small) || std::get<1>(k) != std::get<1>(small) ||
            std::get<3>(k) != std::get<3>(small) || std::get<4>(k) != std::get<4>(small))
          continue;
        if (lds[k] < lds[small] || waves[k] < waves[small]) continue;
        if (!into || waves[k] > waves[*into]) into = &kv.first;
      }
      if (!into) continue;
      const Key target = *into;
      std::vector<int>& dst = cls[target];
      dst.insert(dst.end(), cls[small].begin(), cls[small].end());
      waves[target] += waves[small];
      cls.erase(small);
    }
  }
  std::vector<double> cost(jobs.size());
  for (size_t k = 0; k < jobs.size(); ++k) {
    const SchedJob& j = jobs[k];
    // a search whose pose is shared by wpp waves takes about 1/wpp of the time
    const double ls_eval = (j.ls_method == kLsSolisWets ? kEnergyOnlyCost : 1.0) / std::max(1, j.L->wpp);
    cost[k] = eval_cost(*j.L) * (1.0 + (j.n_ls > 0 ? ls_eval * (double)j.ls_iters : 0.0));
  }
  for (auto& kv : cls) {
    std::vector<int>& m = kv.second;
    std::stable_sort(m.begin(), m.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    ClassChain c{};
    c.A = std::get<0>(kv.first);
    c.wpb = std::get<1>(kv.first);
    c.ls_method = std::get<3>(kv.first);
    c.wpp = std::get<4>(kv.first);
    c.pop_first = (int)out.blocks.size();
    for (int k : m) {
      const SchedJob& j = jobs[k];
      const long long waves = (long long)j.n_runs * j.pop_size;
      for (long long w = 0; w < waves; w += c.wpb) out.blocks.push_back(make_int2(j.slot, (int)w));
      c.lds = std::max(c.lds, j.L->lds_bytes);
      c.latency = std::max(c.latency, cost[k]);
    }
    c.pop_count = (int)out.blocks.size() - c.pop_first;
    c.ls_first = (int)out.blocks.size();
    const int searches_per_block = std::max(1, c.wpb / c.wpp);
    for (int k : m) {
      const SchedJob& j = jobs[k];
      const long long searches = (long long)j.n_runs * j.n_ls;
      for (long long w = 0; w < searches; w += searches_per_block) out.blocks.push_back(make_int2(j.slot, (int)w));
    }
    c.ls_count = (int)out.blocks.size() - c.ls_first;
    c.run_first = (int)out.blocks.size();
    for (int k : m) {
      const SchedJob& j = jobs[k];
      if (j.n_ls > 0)
        for (int r = 0; r < j.n_runs; r += kWavesPerBlock) out.blocks.push_back(make_int2(j.slot, r));
    }
    c.run_count = (int)out.blocks.size() - c.run_first;
    c.adv_first = (int)out.blocks.size();
    for (int k : m) out.blocks.push_back(make_int2(jobs[k].slot, 0));
    c.adv_count = (int)out.blocks.size() - c.adv_first;
    out.classes.push_back(c);
  }
  double slowest = 0.0;
  for (const ClassChain& c : out.classes) slowest = std::max(slowest, c.latency);
  for (ClassChain& c : out.classes) {
    if (max_reps <= 0) {
      c.reps = std::max(1, uniform_reps);
    } else {
      const double r = c.latency > 0.0 ? std::floor(slowest / c.latency) : 1.0;
      c.reps = (int)std::max(1.0, std::min((double)max_reps, r));
    }
  }
}

hipError_t launch_init_phase(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                             hipStream_t s, const LaunchHook* hook) {
  for (const ClassChain& c : g.classes) {
    auto f = [&] { return launch_ga_init(table, d_blocks + c.pop_first, c.pop_count, c.A, c.wpb, c.lds, R, s); };
    const hipError_t e = hook ? (*hook)(MD_K_INIT_POPULATION, f) : f();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

// The launch of one phase (kind) of one class's generation on stream st (none where the class
// has no such work).
hipError_t launch_step(const ClassChain& c, int kind, JobDev* table, const int2* d_blocks, const RecDev& R,
                       hipStream_t st) {
  switch (kind) {
    case MD_K_GENERATION:
      return launch_ga_generation(table, d_blocks + c.pop_first, c.pop_count, c.A, c.wpb, c.lds, R, st);
    case MD_K_LS_PICK:
      return c.run_count > 0 ? launch_ga_ls_pick(table, d_blocks + c.run_first, c.run_count, st) : hipSuccess;
    case MD_K_LOCAL_SEARCH:
      return c.ls_count > 0 ? launch_ga_local_search(table, d_blocks + c.ls_first, c.ls_count, c.A, c.wpb, c.wpp,
                                                     c.lds, c.ls_method, R, st)
                            : hipSuccess;
    default:
      return launch_ga_advance_list(table, d_blocks + c.adv_first, c.adv_count, st);
  }
}

constexpr int kChainKinds[4] = {MD_K_GENERATION, MD_K_LS_PICK, MD_K_LOCAL_SEARCH, MD_K_SUM_EVALS};

bool has_step(const ClassChain& c, int kind) {
  return !(kind == MD_K_LS_PICK && c.run_count == 0) && !(kind == MD_K_LOCAL_SEARCH && c.ls_count == 0);
}

// One generation of one class on stream st.
hipError_t launch_chain(const ClassChain& c, JobDev* table, const int2* d_blocks, const RecDev& R, hipStream_t st,
                        const LaunchHook* hook) {
  hipError_t e = hipSuccess;
  for (int kind : kChainKinds) {
    if (e != hipSuccess || !has_step(c, kind)) continue;
    auto f = [&] { return launch_step(c, kind, table, d_blocks, R, st); };
    e = hook ? (*hook)(kind, f) : f();
  }
  return e;
}

}  // namespace

hipError_t launch_generation_phase(const GenSchedule& g, JobDev* table, const int2* d_blocks,
                                   const RecDev& R, hipStream_t s, const LaunchHook* hook) {
  for (const ClassChain& c : g.classes) {
    const hipError_t e = launch_chain(c, table, d_blocks, R, s, hook);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ captured generations
hipError_t GenGraph::make_streams() {
  if (cs_) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking);
  for (size_t k = 0; k + 1 < kGraphBranches && e == hipSuccess; ++k) {
    hipStream_t x = nullptr;
    e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (e == hipSuccess) side_.push_back(x);
  }
  ev_.assign(kGraphBranches, nullptr);
  for (hipEvent_t& x : ev_)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
  if (e != hipSuccess) {
    // all or nothing: a later call starts over instead of finding a partial set
    for (hipEvent_t x : ev_)
      if (x) (void)hipEventDestroy(x);
    for (hipStream_t x : side_) (void)hipStreamDestroy(x);
    if (cs_) (void)hipStreamDestroy(cs_);
    ev_.clear();
    side_.clear();
    cs_ = nullptr;
  }
  return e;
}

GenGraph::~GenGraph() {
  reset();
  for (hipEvent_t x : ev_)
    if (x) (void)hipEventDestroy(x);
  for (hipStream_t x : side_) (void)hipStreamDestroy(x);
  if (cs_) (void)hipStreamDestroy(cs_);
}

hipError_t GenGraph::fork_classes(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                                  hipStream_t main, bool sink) {
  // class i runs on stream i mod width (0 = main); every side stream in use waits for the fork
  // and joins back into main at the end.  With `sink` (capture) an empty kernel on main after
  // the join becomes the graph's only sink: without it each branch's last node is a sink of
  // its own, and nothing but the runtime's handling of several sinks would order work queued
  // after the graph's launch behind the side branches.
  const size_t width = std::max<size_t>(1, std::min(g.classes.size(), kGraphBranches));
  hipError_t e = hipEventRecord(ev_[0], main);
  for (size_t k = 0; k + 1 < width && e == hipSuccess; ++k) e = hipStreamWaitEvent(side_[k], ev_[0], 0);
  for (size_t i = 0; i < g.classes.size() && e == hipSuccess; ++i) {
    const ClassChain& c = g.classes[i];
    hipStream_t st = (i % width == 0) ? main : side_[i % width - 1];
    for (int r = 0; r < c.reps && e == hipSuccess; ++r) e = launch_chain(c, table, d_blocks, R, st, nullptr);
  }
  for (size_t k = 0; k + 1 < width && e == hipSuccess; ++k) e = hipEventRecord(ev_[1 + k], side_[k]);
  for (size_t k = 0; k + 1 < width && e == hipSuccess; ++k) e = hipStreamWaitEvent(main, ev_[1 + k], 0);
  if (e == hipSuccess && sink) e = launch_join(main);
  return e;
}

hipError_t GenGraph::capture(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R) {
  reset();
  hipError_t e = make_streams();
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t el = fork_classes(g, table, d_blocks, R, cs_, true);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs_, &graph);
  if (e == hipSuccess) e = el;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess && exec_) {
    (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
  }
  return e;
}

hipError_t GenGraph::launch_direct(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                                   hipStream_t s) {
  const hipError_t e = make_streams();
  return e == hipSuccess ? fork_classes(g, table, d_blocks, R, s, false) : e;
}

hipError_t GenGraph::launch_phased(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                                   hipStream_t s, const LaunchHook* hook) {
  hipError_t e = make_streams();
  const size_t width = std::max<size_t>(1, std::min(g.classes.size(), kGraphBranches));
  for (int kind : kChainKinds) {
    if (e != hipSuccess) break;
    bool any = false;
    for (const ClassChain& c : g.classes) any = any || has_step(c, kind);
    if (!any) continue;
    auto phase = [&]() -> hipError_t {
      hipError_t ep = hipEventRecord(ev_[0], s);
      for (size_t k = 0; k + 1 < width && ep == hipSuccess; ++k) ep = hipStreamWaitEvent(side_[k], ev_[0], 0);
      for (size_t i = 0; i < g.classes.size() && ep == hipSuccess; ++i)
        if (has_step(g.classes[i], kind))
          ep = launch_step(g.classes[i], kind, table, d_blocks, R, (i % width == 0) ? s : side_[i % width - 1]);
      for (size_t k = 0; k + 1 < width && ep == hipSuccess; ++k) ep = hipEventRecord(ev_[1 + k], side_[k]);
      for (size_t k = 0; k + 1 < width && ep == hipSuccess; ++k) ep = hipStreamWaitEvent(s, ev_[1 + k], 0);
      return ep;
    };
    e = hook ? (*hook)(kind, phase) : phase();
  }
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
