// Autotuner for the per-ligand launch plan of libmdock (md_ligand_autotune, md_ligand_set_plan,
// md_ligand_get_plan, md_tune_table_clear in include/mdock.h).
//
// The evaluation kernels' tile and schedule choices for a ligand are: how many poses (waves)
// share a block, how much LDS a block takes (which sets how many pair rows are staged in LDS
// rather than read from global memory, and how many blocks fit on a compute unit), and the size
// of the conflict-free lane groups of the pair schedule (which sets the number of force-array
// copies).  Which combination is fastest depends on the ligand's size and on the device, so it is
// measured: the local-search kernel runs on the caller's receptor for every candidate plan, and
// the fastest is kept in the ligand and in a process-wide table keyed by the ligand's size class,
// from which later ligands of that class take their plan when they are created.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "internal.h"
#include "mdock.h"

namespace mdock {
md_status api_fail(md_status st, const std::string& msg);
md_status api_hip_fail(hipError_t e, const std::string& what);
}  // namespace mdock

using namespace mdock;

namespace {

constexpr int kFillStarts = 8192;   // local searches that fill the device several times over

// Size class: atoms per lane and a quarter-octave bucket of the pair count.
std::pair<int, int> size_class(const LigHost& h) {
  const int A = h.n_atoms > kWave ? 2 : 1;
  return {A, (int)std::floor(4.0 * std::log2((double)h.n_pairs + 1.0))};
}

struct TuneEntry {
  PlanParams plan;
  double us_per_eval;
};

std::mutex g_table_mu;
std::map<std::pair<int, int>, TuneEntry> g_table;

bool valid_plan(const md_plan& p) {
  return p.lds_budget >= 0 && p.lds_budget <= kMaxLdsPerBlock && p.group_div >= 2 && p.group_div <= 8 &&
         (p.waves_per_block == 1 || p.waves_per_block == 2 || p.waves_per_block == 4 ||
          p.waves_per_block == 8 || p.waves_per_block == 12 || p.waves_per_block == 16) &&
         (p.waves_per_pose == 0 || p.waves_per_pose == 1 || p.waves_per_pose == 2 || p.waves_per_pose == 4);
}

PlanParams to_params(const md_plan& p) {
  PlanParams pp;
  pp.lds_budget = p.lds_budget;
  pp.group_div = p.group_div;
  pp.wpb = p.waves_per_block;
  pp.wpp = std::max(1, p.waves_per_pose);
  return pp;
}

void describe(const LigHost& h, md_plan* out) {
  out->lds_budget = h.plan.lds_budget;
  out->group_div = h.plan.group_div;
  out->waves_per_block = h.wpb;
  out->waves_per_pose = h.wpp;
  out->lds_bytes = h.lds_bytes;
  out->staged_rows = h.pl_rows;
  out->total_rows = h.n_rows;
}

// Re-plans the ligand and swaps its device buffer (the old one is freed once the device is idle).
hipError_t apply_plan(md_ligand* l, const PlanParams& pp) {
  LigHost h = l->host;
  plan_ligand(h, pp);
  if (h.lds_bytes > kMaxLdsPerBlock) return hipErrorInvalidValue;
  void* buf = nullptr;
  LigDev L{};
  hipError_t e = upload_ligand(h, &buf, &L);
  if (e != hipSuccess) return e;
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return e;
  }
  (void)hipFree(l->d_buf);
  l->d_buf = buf;
  l->dev = L;
  l->host = std::move(h);
  return hipSuccess;
}

// Random start genotypes inside the receptor box (tuning input only; fixed seed).
std::vector<float> tuning_genes(const RecDev& R, int n_genes, int n) {
  std::mt19937_64 rng(0x5eedull);
  std::uniform_real_distribution<float> u(0.f, 1.f);
  std::vector<float> g((size_t)n * n_genes);
  const float ext[3] = {(R.nx - 1) * R.h, (R.ny - 1) * R.h, (R.nz - 1) * R.h};
  const float org[3] = {R.ox, R.oy, R.oz};
  for (int k = 0; k < n; ++k) {
    float* x = &g[(size_t)k * n_genes];
    for (int a = 0; a < 3; ++a) x[a] = org[a] + ext[a] * (0.25f + 0.5f * u(rng));
    float q[4], s = 0.f;
    for (float& c : q) {
      c = 2.f * u(rng) - 1.f;
      s += c * c;
    }
    s = std::sqrt(std::max(s, 1e-12f));
    for (int a = 0; a < 4; ++a) x[3 + a] = q[a] / s;
    for (int a = 7; a < n_genes; ++a) x[a] = 3.14159265f * (2.f * u(rng) - 1.f);
  }
  return g;
}

struct Bench {
  const RecDev* R;
  hipStream_t s;
  int n, iters;
  float *genes_in, *genes_out, *energy;
  hipEvent_t a, b;
  // microseconds per evaluation (best of five launches after one warm-up), or < 0 on error
  double time(const LigDev& L, hipError_t* err) {
    double best = 1e300;
    for (int rep = 0; rep < 6; ++rep) {
      hipError_t e = hipEventRecord(a, s);
      if (e == hipSuccess)
        e = launch_local_search(L, *R, n, genes_in, genes_out, energy, iters, 0.8f, 0.01f, nullptr, nullptr, nullptr, s);
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) {
        *err = e;
        return -1.0;
      }
      if (rep > 0) best = std::min(best, (double)ms * 1e3 / ((double)n * iters));
    }
    return best;
  }
};

}  // namespace


extern "C" {

md_status md_ligand_get_plan(const md_ligand* lig, md_plan* out) {
  if (!lig || !out) return api_fail(MD_EINVAL, "md_ligand_get_plan: null argument");
  describe(lig->host, out);
  return MD_OK;
}

md_status md_ligand_set_plan(md_ligand* lig, const md_plan* plan) {
  if (!lig || !plan) return api_fail(MD_EINVAL, "md_ligand_set_plan: null argument");
  if (lig->holds.load() > 0) return api_fail(MD_EBUSY, "md_ligand_set_plan: a server request still uses the ligand");
  if (!valid_plan(*plan))
    return api_fail(MD_ERANGE, "md_ligand_set_plan: lds_budget in [0, 163840], group_div in [2, 8], "
                               "waves_per_block in {1, 2, 4, 8, 12, 16}, waves_per_pose in {1, 2, 4}");
  LigHost probe = lig->host;
  plan_ligand(probe, to_params(*plan));
  if (probe.lds_bytes > kMaxLdsPerBlock)
    return api_fail(MD_ERANGE, "md_ligand_set_plan: the plan needs more than 160 KiB of LDS per block");
  hipError_t e = apply_plan(lig, to_params(*plan));
  if (e != hipSuccess) return api_hip_fail(e, "md_ligand_set_plan");
  return MD_OK;
}

md_status md_schedule_preview(const md_ligand_desc* d, md_plan* plan, unsigned* pair_slots, int capacity,
                              int* group_lanes) {
  if (!d || !plan) return api_fail(MD_EINVAL, "md_schedule_preview: null argument");
  if (!valid_plan(*plan))
    return api_fail(MD_ERANGE, "md_schedule_preview: lds_budget in [0, 163840], group_div in [2, 8], "
                               "waves_per_block in {1, 2, 4, 8, 12, 16}, waves_per_pose in {1, 2, 4}");
  LigHost h;
  bool range = false;
  const std::string err = prepare_ligand(d->n_atoms, d->xyz, d->type, d->charge, d->n_bonds, d->bonds,
                                         d->n_torsions, d->torsions, d->root_atom, d->n_types,
                                         d->type_params, h, range);
  if (!err.empty()) return api_fail(range ? MD_ERANGE : MD_EINVAL, "md_schedule_preview: " + err);
  plan_ligand(h, to_params(*plan));
  if (h.lds_bytes > kMaxLdsPerBlock)
    return api_fail(MD_ERANGE, "md_schedule_preview: the plan needs more than 160 KiB of LDS per block");
  describe(h, plan);
  if (pair_slots && capacity > 0) {
    const size_t k = std::min<size_t>((size_t)capacity, h.pair_ij.size());
    std::memcpy(pair_slots, h.pair_ij.data(), k * sizeof(unsigned));
  }
  if (group_lanes) *group_lanes = h.group_lanes;
  return MD_OK;
}

md_status md_tune_table_clear(void) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  g_table.clear();
  return MD_OK;
}

int md_tune_table_size(void) {
  std::lock_guard<std::mutex> lk(g_table_mu);
  return (int)g_table.size();
}

md_status md_ligand_autotune(const md_receptor* rec, md_ligand* lig, int n_starts, int flags,
                             void* hip_stream, md_tune_info* info) {
  if (!rec || !lig) return api_fail(MD_EINVAL, "md_ligand_autotune: null handle");
  if (lig->holds.load() > 0) return api_fail(MD_EBUSY, "md_ligand_autotune: a server request still uses the ligand");
  if (flags & ~MD_TUNE_FORCE) return api_fail(MD_EINVAL, "md_ligand_autotune: unknown flags");
  if (n_starts < 0 || n_starts > (1 << 20)) return api_fail(MD_ERANGE, "md_ligand_autotune: n_starts in [0, 2^20]");
  md_tune_info out{};
  const std::pair<int, int> cls = size_class(lig->host);
  // the table holds plans for full-device launches (batches and servers); a plan for a given,
  // smaller launch is tuned for that launch and kept in the ligand only
  const bool fill = n_starts == 0 || n_starts >= kFillStarts;
  if (fill && !(flags & MD_TUNE_FORCE)) {
    TuneEntry hit{};
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_table_mu);
      auto it = g_table.find(cls);
      if (it != g_table.end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found) {
      hipError_t e = apply_plan(lig, hit.plan);
      if (e != hipSuccess) return api_hip_fail(e, "md_ligand_autotune");
      describe(lig->host, &out.plan);
      out.us_per_eval = hit.us_per_eval;
      out.from_table = 1;
      if (info) *info = out;
      return MD_OK;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const RecDev& R = rec->dev;
  const LigHost base = lig->host;
  // the launch size to tune for; enough steps for ~1 ms per launch
  const int n = fill ? kFillStarts : n_starts;
  const double slots = (double)base.n_rows * kWave + 64.0;
  const int iters = (int)std::max(2.0, std::min(300.0, std::round(8e7 / (n * slots))));
  const std::vector<float> g = tuning_genes(R, base.n_genes, n);
  Bench bench{&R, s, n, iters, nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t gb = g.size() * sizeof(float);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&bench.genes_in), gb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&bench.genes_out), gb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&bench.energy), (size_t)n * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(bench.genes_in, g.data(), gb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&bench.a);
  if (e == hipSuccess) e = hipEventCreate(&bench.b);

  // candidates: first waves per block x LDS budget (lane groups ~N/3), then the lane-group size
  // for the best of those; plans that come out identical are timed once
  struct Cand {
    PlanParams pp;
    double us;
  };
  std::vector<Cand> tried;
  auto same_plan = [](const LigHost& x, const LigHost& y) {
    return x.wpb == y.wpb && x.wpp == y.wpp && x.pl_rows == y.pl_rows && x.group_lanes == y.group_lanes &&
           x.lds_bytes == y.lds_bytes;
  };
  std::vector<LigHost> plans_seen;
  auto try_plan = [&](const PlanParams& pp) -> double {
    LigHost h = base;
    plan_ligand(h, pp);
    if (h.lds_bytes > kMaxLdsPerBlock) return -1.0;
    for (size_t k = 0; k < plans_seen.size(); ++k)
      if (same_plan(plans_seen[k], h)) return tried[k].us;
    void* buf = nullptr;
    LigDev L{};
    hipError_t ee = upload_ligand(h, &buf, &L);
    double us = -1.0;
    if (ee == hipSuccess) us = bench.time(L, &ee);
    if (buf) {
      hipError_t es = hipStreamSynchronize(s);
      if (ee == hipSuccess) ee = es;
      (void)hipFree(buf);
    }
    if (ee != hipSuccess) {
      e = ee;
      return -1.0;
    }
    plans_seen.push_back(h);
    tried.push_back({pp, us});
    return us;
  };
  PlanParams best = base.plan;
  double best_us = 1e300, default_us = -1.0;
  if (e == hipSuccess) {
    default_us = try_plan(PlanParams());
    if (default_us > 0) {
      best = PlanParams();
      best_us = default_us;
    }
  }
  const int budgets[] = {32 * 1024, 48 * 1024, 64 * 1024, 96 * 1024, 128 * 1024, kMaxLdsPerBlock};
  const int wide = max_waves_per_block(base.n_atoms > kWave ? 2 : 1);
  for (int wpb : {4, 8, wide})
    for (int budget : budgets) {
      // the widest blocks (one per compute unit) only with the large budgets
      if (wpb == wide && budget < 96 * 1024) continue;
      if (e != hipSuccess) break;
      PlanParams pp;
      pp.wpb = wpb;
      pp.lds_budget = budget;
      const double us = try_plan(pp);
      if (us > 0 && us < best_us) {
        best_us = us;
        best = pp;
      }
    }
  for (int wpp : {2, 4})
    for (int budget : {64 * 1024, kMaxLdsPerBlock}) {
      if (e != hipSuccess) break;
      PlanParams pp;
      pp.wpp = wpp;
      pp.wpb = wpp;
      pp.lds_budget = budget;
      const double us = try_plan(pp);
      if (us > 0 && us < best_us) {
        best_us = us;
        best = pp;
      }
    }
  for (int div : {2, 4}) {
    if (e != hipSuccess) break;
    PlanParams pp = best;
    pp.group_div = div;
    const double us = try_plan(pp);
    if (us > 0 && us < best_us) {
      best_us = us;
      best = pp;
    }
  }
  if (bench.a) (void)hipEventDestroy(bench.a);
  if (bench.b) (void)hipEventDestroy(bench.b);
  if (bench.genes_in) (void)hipFree(bench.genes_in);
  if (bench.genes_out) (void)hipFree(bench.genes_out);
  if (bench.energy) (void)hipFree(bench.energy);
  if (e != hipSuccess) return api_hip_fail(e, "md_ligand_autotune");
  e = apply_plan(lig, best);
  if (e != hipSuccess) return api_hip_fail(e, "md_ligand_autotune");
  if (fill) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_table[cls] = TuneEntry{best, best_us};
  }
  describe(lig->host, &out.plan);
  out.us_per_eval = best_us;
  out.default_us_per_eval = default_us;
  out.candidates = (int)tried.size();
  out.from_table = 0;
  if (info) *info = out;
  return MD_OK;
}

// Batch autotuner.  A batch mixes ligand sizes in shared launches (one per size class and phase,
// in parallel graph branches), so the plan that is fastest for a ligand alone on the whole device
// need not be fastest in the mix.  Here whole-batch plan policies are timed on the batch itself,
// for a few generations each, and the fastest is applied to every ligand.
md_status md_batch_autotune(const md_receptor* rec, int n, md_ligand* const* ligands,
                            const md_dock_params* params, int generations, void* hip_stream,
                            md_batch_tune_info* info) {
  if (!rec || n < 1 || !ligands || !params) return api_fail(MD_EINVAL, "md_batch_autotune: null argument");
  if (generations < 2 || generations > 1000) return api_fail(MD_ERANGE, "md_batch_autotune: generations in [2, 1000]");
  for (int k = 0; k < n; ++k) {
    if (!ligands[k]) return api_fail(MD_EINVAL, "md_batch_autotune: null ligand");
    if (ligands[k]->holds.load() > 0)
      return api_fail(MD_EBUSY, "md_batch_autotune: a server request still uses ligand " + std::to_string(k));
  }
  // scratch results and shortened searches: each policy is timed at g1 and at g2 generations and
  // charged (t2 - t1) / (g2 - g1) per generation, which leaves out the per-call costs
  // (workspace, schedule, graph capture, initial population)
  const int g2 = std::max(2, generations), g1 = std::max(1, g2 / 3);
  std::vector<md_dock_params> P(params, params + n);
  for (auto& p : P) p.max_evals_per_run = (long long)1 << 62;
  std::vector<std::vector<float>> be(n), bg(n);
  std::vector<md_dock_result> res(n);
  std::vector<md_dock_job> jobs(n);
  for (int k = 0; k < n; ++k) {
    be[k].resize(P[k].n_runs);
    bg[k].resize((size_t)P[k].n_runs * ligands[k]->dev.n_genes);
    res[k] = md_dock_result{};
    res[k].n_runs = P[k].n_runs;
    res[k].n_genes = ligands[k]->dev.n_genes;
    res[k].n_atoms = ligands[k]->dev.n_atoms;
    res[k].best_energy = be[k].data();
    res[k].best_genes = bg[k].data();
    jobs[k] = md_dock_job{ligands[k], P[k], &res[k]};
  }
  auto apply_all = [&](const std::vector<PlanParams>& plans) -> md_status {
    for (int k = 0; k < n; ++k) {
      LigHost probe = ligands[k]->host;
      plan_ligand(probe, plans[k]);
      if (probe.lds_bytes > kMaxLdsPerBlock) continue;   // keep the ligand's current plan
      hipError_t e = apply_plan(ligands[k], plans[k]);
      if (e != hipSuccess) return api_hip_fail(e, "md_batch_autotune");
    }
    return MD_OK;
  };
  auto run = [&](int gens, double* ms) -> md_status {
    for (int k = 0; k < n; ++k) jobs[k].params.max_generations = gens;
    const auto t0 = std::chrono::steady_clock::now();
    const md_status st = md_dock_batch(rec, n, jobs.data(), hip_stream);
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
  };
  // the shorter of two runs at each length, after a warm-up (first use of the plans)
  auto time_batch = [&](double* ms) -> md_status {
    double t1 = 1e300, t2 = 1e300, t = 0.0;
    md_status st = run(g1, &t);
    for (int rep = 0; rep < 2 && st == MD_OK; ++rep) {
      st = run(g1, &t);
      t1 = std::min(t1, t);
      if (st == MD_OK) st = run(g2, &t);
      t2 = std::min(t2, t);
    }
    *ms = std::max(t2 - t1, 1e-6) / (g2 - g1);
    return st;
  };
  const int n_pol = MD_BATCH_POLICIES;
  std::vector<std::vector<PlanParams>> plans(n_pol, std::vector<PlanParams>(n));
  for (int k = 0; k < n; ++k) {
    plans[MD_POLICY_LDS_ALL][k].lds_budget = kMaxLdsPerBlock;
    plans[MD_POLICY_WIDE_BLOCKS][k].wpb = 8;
    plans[MD_POLICY_SMALL_GROUPS][k].group_div = 2;
    plans[MD_POLICY_FULL_BLOCKS][k].wpb = max_waves_per_block(ligands[k]->host.n_atoms > kWave ? 2 : 1);
    plans[MD_POLICY_FULL_BLOCKS][k].lds_budget = kMaxLdsPerBlock;
    if (ligands[k]->host.n_atoms > kWave) {
      plans[MD_POLICY_SHARED_LARGE][k].wpp = 4;
      plans[MD_POLICY_SHARED_LARGE][k].wpb = 4;
    }
  }
  md_batch_tune_info out{};
  out.n_policies = n_pol;
  double best = 1e300;
  for (int pol = 0; pol < n_pol; ++pol) {
    md_status st = MD_OK;
    if (pol == MD_POLICY_TUNED_ALONE) {
      for (int k = 0; k < n && st == MD_OK; ++k) {
        st = md_ligand_autotune(rec, ligands[k], 0, 0, hip_stream, nullptr);
        plans[pol][k] = ligands[k]->host.plan;
      }
    } else {
      st = apply_all(plans[pol]);
    }
    double ms = 0.0;
    if (st == MD_OK) st = time_batch(&ms);
    if (st != MD_OK) return st;
    out.ms_per_generation[pol] = ms;
    if (ms < best) {
      best = ms;
      out.policy = pol;
    }
  }
  md_status st = apply_all(plans[out.policy]);
  if (st != MD_OK) return st;
  if (info) *info = out;
  return MD_OK;
}

}  // extern "C"

