// md_dock_noalloc (include/mdock.h): md_dock without any device allocation, for callers that
// cannot allocate.  The dock's workspace -- job table, block table, both population buffers,
// energies, evaluation counts, local-search picks and the per-run results -- lives in `scratch`,
// a file-scope device array of kScratchBytes that every GPU the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel or a copy: the name is only
// a host-side stand-in.  The array's device address is looked up once per device (with that
// device current) through hipGetSymbolAddress and kept; every use goes through that pointer.
// Calls that overlap on one GPU share the array and race; a call leaves its workspace behind,
// and the next call rewrites every part it reads before reading it (the job table and block
// table are uploaded, the populations and results are written by the kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mdock.h"

namespace mdock {
md_status api_fail(md_status st, const std::string& msg);
md_status api_hip_fail(hipError_t e, const std::string& what);
int n_local_search_of(const md_dock_params* p);
std::string check_dock_params(const md_dock_params* p);
}  // namespace mdock

using namespace mdock;

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;   // 8 MiB per device
constexpr int kMaxDevices = 64;
constexpr int kMaxRunsNoAlloc = 1024;               // the host-side order of runs lives on the stack

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (looked up on the device's first call).
hipError_t scratch_on_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return hipSuccess;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

extern "C" {

md_status md_dock_noalloc(const md_receptor* rec, const md_ligand* lig, const md_dock_params* p,
                          md_dock_result* out, void* hip_stream) {
  if (!rec || !lig || !p || !out) return api_fail(MD_EINVAL, "md_dock_noalloc: null argument");
  const std::string err = check_dock_params(p);
  if (!err.empty()) {
    const bool range = err.find("<=") != std::string::npos || err.find("too large") != std::string::npos;
    return api_fail(range ? MD_ERANGE : MD_EINVAL, "md_dock_noalloc: " + err);
  }
  const LigDev& L = lig->dev;
  const int runs = p->n_runs, G = L.n_genes, N = L.n_atoms;
  if (out->n_runs < runs || out->n_genes < G || !out->best_energy || !out->best_genes)
    return api_fail(MD_EINVAL, "md_dock_noalloc: result buffers too small or null");
  if (out->best_xyz && out->n_atoms < N) return api_fail(MD_EINVAL, "md_dock_noalloc: best_xyz capacity too small");
  if (runs > kMaxRunsNoAlloc)
    return api_fail(MD_ERANGE, "md_dock_noalloc: n_runs must be <= " + std::to_string(kMaxRunsNoAlloc));

  // workspace layout inside the scratch array
  const int n_ls = n_local_search_of(p);
  const size_t rows = (size_t)runs * p->pop_size;
  std::vector<SchedJob> sj{SchedJob{0, &L, runs, p->pop_size, n_ls, p->ls_iters, p->ls_method}};
  GenSchedule sched;
  build_schedule(sj, sched, 0, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_table = take(sizeof(JobDev));
  const size_t o_blocks = take(sizeof(int2) * std::max<size_t>(sched.blocks.size(), 1));
  const size_t o_ga = take(rows * G * 4), o_gb = take(rows * G * 4);
  const size_t o_ea = take(rows * 4), o_eb = take(rows * 4), o_ev = take(rows * 4);
  const size_t o_lsr = take((size_t)runs * std::max(n_ls, 1) * 4), o_br = take((size_t)runs * 4);
  const size_t o_be = take((size_t)runs * 4), o_bg = take((size_t)runs * G * 4), o_er = take((size_t)runs * 8);
  const size_t o_bx = out->best_xyz ? take((size_t)runs * N * 12) : 0;
  if (off > kScratchBytes)
    return api_fail(MD_ERANGE, "md_dock_noalloc: the dock needs " + std::to_string(off) +
                                   " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                   " bytes of the static scratch array (fewer runs or a smaller population)");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  char* w = nullptr;
  if (e == hipSuccess) e = scratch_on_device(dev, &w);
  if (e != hipSuccess) return api_hip_fail(e, "md_dock_noalloc: scratch array");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);

  JobDev J{};
  J.L = L;
  GaDev& P = J.P;
  P.n_runs = runs;
  P.pop_size = p->pop_size;
  P.n_genes = G;
  P.n_ls = n_ls;
  P.ls_iters = p->ls_iters;
  P.ls_method = p->ls_method;
  P.elitism = p->elitism;
  P.rho = p->rho;
  P.eps = p->eps;
  P.crossover_rate = p->crossover_rate;
  P.mutation_rate = p->mutation_rate;
  P.tournament_rate = p->tournament_rate;
  P.mut_trans = p->mut_trans;
  P.mut_rot = p->mut_rot;
  P.mut_tors = p->mut_tors;
  P.seed = p->seed;
  J.genes[0] = reinterpret_cast<float*>(w + o_ga);
  J.genes[1] = reinterpret_cast<float*>(w + o_gb);
  J.energy[0] = reinterpret_cast<float*>(w + o_ea);
  J.energy[1] = reinterpret_cast<float*>(w + o_eb);
  J.evals = reinterpret_cast<int*>(w + o_ev);
  J.evals_of_runs = reinterpret_cast<long long*>(w + o_er);
  J.ls_rows = reinterpret_cast<int*>(w + o_lsr);
  J.best_row = reinterpret_cast<int*>(w + o_br);
  J.best_energy = reinterpret_cast<float*>(w + o_be);
  J.best_genes = reinterpret_cast<float*>(w + o_bg);
  J.best_xyz = out->best_xyz ? reinterpret_cast<float*>(w + o_bx) : nullptr;
  J.gen = 0;
  J.cur = 0;
  J.planned = md_dock_planned_generations(p);
  J.state = kJobInit;
  JobDev* d_table = reinterpret_cast<JobDev*>(w + o_table);
  int2* d_blocks = reinterpret_cast<int2*>(w + o_blocks);

  // every generation kernel by kernel on the caller's stream (no graph: instantiating one
  // allocates); the epilogue that finished each run wrote its best genes, energy and pose
  e = hipMemcpyAsync(d_table, &J, sizeof(JobDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !sched.blocks.empty())
    e = hipMemcpyAsync(d_blocks, sched.blocks.data(), sizeof(int2) * sched.blocks.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_init_phase(sched, d_table, d_blocks, rec->dev, s, nullptr);
  if (e == hipSuccess) e = launch_ga_advance(d_table, 1, s);
  for (int g = 1; g <= J.planned && e == hipSuccess; ++g)
    e = launch_generation_phase(sched, d_table, d_blocks, rec->dev, s, nullptr);
  // results straight into the caller's rows (row strides are the caller's capacities), then
  // sorted by energy on the host in place
  if (e == hipSuccess)
    e = hipMemcpyAsync(out->best_energy, w + o_be, (size_t)runs * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(out->best_genes, (size_t)out->n_genes * 4, w + o_bg, (size_t)G * 4, (size_t)G * 4, runs,
                         hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && out->best_xyz)
    e = hipMemcpy2DAsync(out->best_xyz, (size_t)out->n_atoms * 12, w + o_bx, (size_t)N * 12, (size_t)N * 12, runs,
                         hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && out->evals)
    e = hipMemcpyAsync(out->evals, w + o_er, (size_t)runs * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return api_hip_fail(e, "md_dock_noalloc");

  // order of the runs by energy (ties: lower run), then each array permuted in place by cycles
  int order[kMaxRunsNoAlloc];
  for (int k = 0; k < runs; ++k) order[k] = k;
  std::stable_sort(order, order + runs, [&](int a, int b) { return out->best_energy[a] < out->best_energy[b]; });
  bool seen[kMaxRunsNoAlloc] = {};
  alignas(8) float row[3 * kMaxAtoms];
  auto permute = [&](auto* base, size_t stride, size_t count) {
    // position k receives original row order[k]
    std::fill(seen, seen + runs, false);
    for (int k = 0; k < runs; ++k) {
      if (seen[k] || order[k] == k) {
        seen[k] = true;
        continue;
      }
      using T = std::remove_pointer_t<decltype(base)>;
      T* tmp = reinterpret_cast<T*>(row);
      std::memcpy(tmp, base + (size_t)k * stride, count * sizeof(T));
      int dst = k;
      while (true) {
        seen[dst] = true;
        const int src = order[dst];
        if (src == k) {
          std::memcpy(base + (size_t)dst * stride, tmp, count * sizeof(T));
          break;
        }
        std::memcpy(base + (size_t)dst * stride, base + (size_t)src * stride, count * sizeof(T));
        dst = src;
      }
    }
  };
  permute(out->best_energy, 1, 1);
  permute(out->best_genes, (size_t)out->n_genes, (size_t)G);
  if (out->best_xyz) permute(out->best_xyz, (size_t)out->n_atoms * 3, (size_t)N * 3);
  if (out->evals) permute(out->evals, 1, 1);
  for (int k = 0; k < runs; ++k) {
    if (out->run_index) out->run_index[k] = order[k];
    if (out->generations) out->generations[k] = J.planned;
  }
  return MD_OK;
}

}  // extern "C"
