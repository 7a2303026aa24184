// C ABI of libmdock (declared in include/mdock.h): handles, validation, error reporting and
// the docking driver that sequences the GA kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "mdock.h"

using namespace mdock;

struct md_receptor {
  RecDev dev{};
  void* d_maps = nullptr;
  int device = 0;
};

struct md_ligand {
  LigDev dev{};
  void* d_buf = nullptr;
  LigHost host;
  int device = 0;
};

namespace {

thread_local std::string g_error;

md_status fail(md_status st, const std::string& msg) {
  g_error = msg;
  return st;
}

md_status hip_fail(hipError_t e, const char* what) {
  g_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? MD_ENOMEM : MD_EDEVICE;
}

#define MD_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

uint16_t f32_to_f16_rne(float f) {
  const _Float16 h = (_Float16)f;   // IEEE conversion, round to nearest even
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Optional per-kernel timing of md_dock's launches (HIP events on the dock's stream).
struct Profiler {
  bool on = false;
  double total_ms[MD_K_COUNT] = {};
  long long launches[MD_K_COUNT] = {};
};
Profiler g_prof;

struct LaunchTimer {
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  hipStream_t s;
  explicit LaunchTimer(hipStream_t st) : s(st) {}
  // brackets one launch; returns the launch's status
  template <typename F>
  hipError_t run(int kind, F&& launch) {
    if (!g_prof.on) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (a && b) marks.push_back({kind, {a, b}});
    else {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
    return e;
  }
  // after the stream has synchronised
  void collect(bool ok) {
    for (auto& m : marks) {
      float ms = 0.f;
      if (ok && hipEventElapsedTime(&ms, m.second.first, m.second.second) == hipSuccess) {
        g_prof.total_ms[m.first] += ms;
        g_prof.launches[m.first] += 1;
      }
      (void)hipEventDestroy(m.second.first);
      (void)hipEventDestroy(m.second.second);
    }
    marks.clear();
  }
};

int n_local_search(const md_dock_params* p) {
  double v = std::ceil((double)p->ls_rate * (double)p->pop_size - 1e-4);
  return (int)std::max(0.0, std::min((double)p->pop_size, v));
}

}  // namespace

extern "C" {

const char* md_last_error(void) { return g_error.c_str(); }

const char* md_version(void) { return "libmdock 0.1 (gfx950)"; }

md_status md_receptor_create(const md_grid_desc* d, const float* maps, md_map_precision stored,
                             void* hip_stream, md_receptor** out) {
  if (!d || !maps || !out) return fail(MD_EINVAL, "md_receptor_create: null argument");
  if (d->n_types != kTypes) return fail(MD_EINVAL, "md_receptor_create: n_types must be 7");
  if (d->nx < 2 || d->ny < 2 || d->nz < 2) return fail(MD_EINVAL, "md_receptor_create: grid needs >= 2 nodes per axis");
  if (!(d->spacing > 0.f) || !std::isfinite(d->spacing)) return fail(MD_EINVAL, "md_receptor_create: bad spacing");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->origin[a])) return fail(MD_EINVAL, "md_receptor_create: bad origin");
  if (stored != MD_MAP_FP32 && stored != MD_MAP_FP16 && stored != MD_MAP_BF16)
    return fail(MD_EINVAL, "md_receptor_create: bad storage precision");
  const long long nodes = (long long)d->nx * d->ny * d->nz;
  if (nodes > (1ll << 31) / kMaps) return fail(MD_ERANGE, "md_receptor_create: grid too large");
  const long long count = nodes * kMaps;
  for (long long i = 0; i < count; ++i)
    if (!std::isfinite(maps[i])) return fail(MD_EINVAL, "md_receptor_create: non-finite map value");
  if (stored == MD_MAP_FP16)
    for (long long i = 0; i < count; ++i)
      if (std::fabs(maps[i]) > 65504.f) return fail(MD_ERANGE, "md_receptor_create: map value outside FP16 range");

  const size_t elem = stored == MD_MAP_FP32 ? 4 : 2;
  std::vector<uint16_t> half;
  const void* src = maps;
  if (stored != MD_MAP_FP32) {
    half.resize(count);
    for (long long i = 0; i < count; ++i)
      half[i] = stored == MD_MAP_FP16 ? f32_to_f16_rne(maps[i]) : f32_to_bf16_rne(maps[i]);
    src = half.data();
  }
  md_receptor* r = new (std::nothrow) md_receptor();
  if (!r) return fail(MD_ENOMEM, "md_receptor_create: out of host memory");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&r->device);
  if (e == hipSuccess) e = hipMalloc(&r->d_maps, count * elem);
  if (e == hipSuccess) e = hipMemcpyAsync(r->d_maps, src, count * elem, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (r->d_maps) (void)hipFree(r->d_maps);
    delete r;
    return hip_fail(e, "md_receptor_create");
  }
  RecDev& R = r->dev;
  R.nx = d->nx;
  R.ny = d->ny;
  R.nz = d->nz;
  R.precision = (int)stored;
  R.ox = d->origin[0];
  R.oy = d->origin[1];
  R.oz = d->origin[2];
  R.h = d->spacing;
  R.inv_h = 1.0f / d->spacing;
  R.map_stride = nodes;
  R.maps = r->d_maps;
  *out = r;
  return MD_OK;
}

md_status md_receptor_destroy(md_receptor* r) {
  if (!r) return MD_OK;
  if (r->d_maps) (void)hipFree(r->d_maps);
  delete r;
  return MD_OK;
}

md_status md_ligand_create(const md_ligand_desc* d, md_ligand** out) {
  if (!d || !out) return fail(MD_EINVAL, "md_ligand_create: null argument");
  md_ligand* l = new (std::nothrow) md_ligand();
  if (!l) return fail(MD_ENOMEM, "md_ligand_create: out of host memory");
  bool range = false;
  std::string err = prepare_ligand(d->n_atoms, d->xyz, d->type, d->charge, d->n_bonds, d->bonds,
                                   d->n_torsions, d->torsions, d->root_atom, d->n_types,
                                   d->type_params, l->host, range);
  if (!err.empty()) {
    delete l;
    return fail(range ? MD_ERANGE : MD_EINVAL, "md_ligand_create: " + err);
  }
  const LigHost& h = l->host;
  const size_t N = h.n_atoms, T = h.n_tors, P = h.pair_ij.size();
  size_t off = 0;
  const size_t o_p0q = off; off = align16(off + N * sizeof(float4));
  const size_t o_type = off; off = align16(off + N * sizeof(int));
  const size_t o_mask = off; off = align16(off + N * sizeof(uint32_t));
  const size_t o_axis = off; off = align16(off + T * sizeof(float4));
  const size_t o_piv = off; off = align16(off + T * sizeof(float4));
  const size_t o_ab = off; off = align16(off + T * sizeof(int2));
  const size_t o_gene = off; off = align16(off + T * sizeof(int));
  const size_t o_ij = off; off = align16(off + P * sizeof(uint32_t));
  const size_t o_coef = off; off = align16(off + P * sizeof(float4));
  const size_t o_inc = off; off = align16(off + h.inc.size() * sizeof(uint32_t));
  std::vector<char> buf(std::max<size_t>(off, 16), 0);
  auto put = [&](size_t o, const void* p, size_t n) { if (n) std::memcpy(buf.data() + o, p, n); };
  put(o_p0q, h.atom_p0q.data(), N * sizeof(float4));
  put(o_type, h.atom_type.data(), N * sizeof(int));
  put(o_mask, h.atom_mask.data(), N * sizeof(uint32_t));
  put(o_axis, h.tor_axis.data(), T * sizeof(float4));
  put(o_piv, h.tor_pivot.data(), T * sizeof(float4));
  put(o_ab, h.tor_ab.data(), T * sizeof(int2));
  put(o_gene, h.tor_gene.data(), T * sizeof(int));
  put(o_ij, h.pair_ij.data(), P * sizeof(uint32_t));
  put(o_coef, h.pair_coef.data(), P * sizeof(float4));
  put(o_inc, h.inc.data(), h.inc.size() * sizeof(uint32_t));
  hipError_t e = hipGetDevice(&l->device);
  if (e == hipSuccess) e = hipMalloc(&l->d_buf, buf.size());
  if (e == hipSuccess) e = hipMemcpy(l->d_buf, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (l->d_buf) (void)hipFree(l->d_buf);
    delete l;
    return hip_fail(e, "md_ligand_create");
  }
  char* b = static_cast<char*>(l->d_buf);
  LigDev& L = l->dev;
  L.n_atoms = (int)N;
  L.n_tors = (int)T;
  L.n_pairs = (int)P;
  L.n_genes = h.n_genes;
  L.atom_p0q = reinterpret_cast<const float4*>(b + o_p0q);
  L.atom_type = reinterpret_cast<const int*>(b + o_type);
  L.atom_mask = reinterpret_cast<const uint32_t*>(b + o_mask);
  L.tor_axis = reinterpret_cast<const float4*>(b + o_axis);
  L.tor_pivot = reinterpret_cast<const float4*>(b + o_piv);
  L.tor_ab = reinterpret_cast<const int2*>(b + o_ab);
  L.tor_gene = reinterpret_cast<const int*>(b + o_gene);
  L.pair_ij = reinterpret_cast<const uint32_t*>(b + o_ij);
  L.pair_coef = reinterpret_cast<const float4*>(b + o_coef);
  L.inc_width = h.inc_width;
  L.inc_stride = h.inc_stride;
  L.inc = reinterpret_cast<const uint32_t*>(b + o_inc);
  *out = l;
  return MD_OK;
}

md_status md_ligand_destroy(md_ligand* l) {
  if (!l) return MD_OK;
  if (l->d_buf) (void)hipFree(l->d_buf);
  delete l;
  return MD_OK;
}

int md_ligand_num_genes(const md_ligand* l) { return l ? l->dev.n_genes : -1; }
int md_ligand_num_atoms(const md_ligand* l) { return l ? l->dev.n_atoms : -1; }
int md_ligand_num_pairs(const md_ligand* l) { return l ? l->dev.n_pairs : -1; }

md_status md_ligand_info(const md_ligand* l, int* n_atoms, int* n_torsions, int* n_pairs,
                         int* sum_moving) {
  if (!l) return fail(MD_EINVAL, "md_ligand_info: null ligand");
  if (n_atoms) *n_atoms = l->dev.n_atoms;
  if (n_torsions) *n_torsions = l->dev.n_tors;
  if (n_pairs) *n_pairs = l->dev.n_pairs;
  if (sum_moving) {
    int s = 0;
    for (uint32_t m : l->host.atom_mask) s += __builtin_popcount(m);
    *sum_moving = s;
  }
  return MD_OK;
}

md_status md_profile_enable(int on) {
  g_prof.on = on != 0;
  return MD_OK;
}

md_status md_profile_reset(void) {
  for (int k = 0; k < MD_K_COUNT; ++k) {
    g_prof.total_ms[k] = 0.0;
    g_prof.launches[k] = 0;
  }
  return MD_OK;
}

md_status md_profile_read(int kind, double* total_ms, long long* launches) {
  if (kind < 0 || kind >= MD_K_COUNT) return fail(MD_EINVAL, "md_profile_read: bad kernel kind");
  if (total_ms) *total_ms = g_prof.total_ms[kind];
  if (launches) *launches = g_prof.launches[kind];
  return MD_OK;
}

md_status md_eval(const md_receptor* rec, const md_ligand* lig, int n_poses, const float* genes,
                  float* energy, float* grad, void* hip_stream) {
  if (!rec || !lig) return fail(MD_EINVAL, "md_eval: null handle");
  if (n_poses < 0) return fail(MD_EINVAL, "md_eval: n_poses < 0");
  if (n_poses == 0) return MD_OK;
  if (!genes || !energy) return fail(MD_EINVAL, "md_eval: null buffer");
  MD_HIP(launch_eval(lig->dev, rec->dev, n_poses, genes, energy, grad,
                     static_cast<hipStream_t>(hip_stream)), "md_eval launch");
  return MD_OK;
}

md_status md_pose(const md_ligand* lig, int n_poses, const float* genes, float* xyz, void* hip_stream) {
  if (!lig) return fail(MD_EINVAL, "md_pose: null handle");
  if (n_poses < 0) return fail(MD_EINVAL, "md_pose: n_poses < 0");
  if (n_poses == 0) return MD_OK;
  if (!genes || !xyz) return fail(MD_EINVAL, "md_pose: null buffer");
  MD_HIP(launch_pose(lig->dev, n_poses, genes, xyz, static_cast<hipStream_t>(hip_stream)), "md_pose launch");
  return MD_OK;
}

md_status md_local_search(const md_receptor* rec, const md_ligand* lig, int n, const float* genes_in,
                          float* genes_out, float* energy_out, int n_iters, float rho, float eps,
                          float* trace, void* hip_stream) {
  if (!rec || !lig) return fail(MD_EINVAL, "md_local_search: null handle");
  if (n < 0) return fail(MD_EINVAL, "md_local_search: n < 0");
  if (n_iters < 1) return fail(MD_EINVAL, "md_local_search: n_iters must be >= 1");
  if (!(rho >= 0.f && rho < 1.f) || !(eps > 0.f) || !std::isfinite(eps))
    return fail(MD_EINVAL, "md_local_search: rho must be in [0,1) and eps > 0");
  if (n == 0) return MD_OK;
  if (!genes_in || !genes_out || !energy_out) return fail(MD_EINVAL, "md_local_search: null buffer");
  MD_HIP(launch_local_search(lig->dev, rec->dev, n, nullptr, genes_in, genes_out, energy_out, nullptr,
                             n_iters, rho, eps, trace, static_cast<hipStream_t>(hip_stream)),
         "md_local_search launch");
  return MD_OK;
}

int md_dock_planned_generations(const md_dock_params* p) {
  if (!p || p->pop_size < 1) return -1;
  const long long per = (long long)(p->pop_size - (p->elitism ? 1 : 0)) +
                        (long long)n_local_search(p) * p->ls_iters;
  long long evals = p->pop_size;
  int gens = 0;
  while (gens < p->max_generations && evals < p->max_evals_per_run) {
    ++gens;
    evals += per;
    if (per <= 0) break;
  }
  return gens;
}

md_status md_dock(const md_receptor* rec, const md_ligand* lig, const md_dock_params* p,
                  md_dock_result* out, void* hip_stream) {
  if (!rec || !lig || !p || !out) return fail(MD_EINVAL, "md_dock: null argument");
  if (p->n_runs < 1 || p->pop_size < 2) return fail(MD_EINVAL, "md_dock: need n_runs >= 1 and pop_size >= 2");
  if (p->pop_size > 1024) return fail(MD_ERANGE, "md_dock: pop_size must be <= 1024");
  if ((long long)p->n_runs * p->pop_size > (1ll << 26)) return fail(MD_ERANGE, "md_dock: n_runs * pop_size too large");
  if (p->elitism != 0 && p->elitism != 1) return fail(MD_EINVAL, "md_dock: elitism must be 0 or 1");
  if (p->max_generations < 0 || p->max_evals_per_run < 0) return fail(MD_EINVAL, "md_dock: negative budget");
  if (!(p->ls_rate >= 0.f && p->ls_rate <= 1.f)) return fail(MD_EINVAL, "md_dock: ls_rate must be in [0,1]");
  const int n_ls = n_local_search(p);
  if (n_ls > 0 && p->ls_iters < 1) return fail(MD_EINVAL, "md_dock: ls_iters must be >= 1");
  if (!(p->rho >= 0.f && p->rho < 1.f) || !(p->eps > 0.f)) return fail(MD_EINVAL, "md_dock: bad rho/eps");
  const float rates[3] = {p->crossover_rate, p->mutation_rate, p->tournament_rate};
  for (float r : rates)
    if (!(r >= 0.f && r <= 1.f)) return fail(MD_EINVAL, "md_dock: rates must be in [0,1]");
  if (!std::isfinite(p->mut_trans) || !std::isfinite(p->mut_rot) || !std::isfinite(p->mut_tors))
    return fail(MD_EINVAL, "md_dock: non-finite mutation size");
  const int G = lig->dev.n_genes, N = lig->dev.n_atoms, runs = p->n_runs, pop = p->pop_size;
  if (out->n_runs < runs || out->n_genes < G || !out->best_energy || !out->best_genes)
    return fail(MD_EINVAL, "md_dock: result buffers too small or null");
  if (out->best_xyz && out->n_atoms < N) return fail(MD_EINVAL, "md_dock: best_xyz capacity too small");

  GaDev P{};
  P.n_runs = runs;
  P.pop_size = pop;
  P.n_genes = G;
  P.n_ls = n_ls;
  P.ls_iters = p->ls_iters;
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
  const int gens = md_dock_planned_generations(p);

  const size_t rows = (size_t)runs * pop;
  size_t off = 0;
  const size_t o_ga = off; off = align16(off + rows * G * 4);
  const size_t o_gb = off; off = align16(off + rows * G * 4);
  const size_t o_ea = off; off = align16(off + rows * 4);
  const size_t o_eb = off; off = align16(off + rows * 4);
  const size_t o_ev = off; off = align16(off + rows * 4);
  const size_t o_er = off; off = align16(off + (size_t)runs * 8);
  const size_t o_ls = off; off = align16(off + (size_t)runs * std::max(n_ls, 1) * 4);
  const size_t o_br = off; off = align16(off + (size_t)runs * 4);
  const size_t o_be = off; off = align16(off + (size_t)runs * 4);
  const size_t o_bg = off; off = align16(off + (size_t)runs * G * 4);
  const size_t o_bx = off; off = align16(off + (size_t)runs * N * 3 * 4);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char* w = nullptr;
  MD_HIP(hipMallocAsync(reinterpret_cast<void**>(&w), off, s), "md_dock workspace");
  float* ga = reinterpret_cast<float*>(w + o_ga);
  float* gb = reinterpret_cast<float*>(w + o_gb);
  float* ea = reinterpret_cast<float*>(w + o_ea);
  float* eb = reinterpret_cast<float*>(w + o_eb);
  int* ev = reinterpret_cast<int*>(w + o_ev);
  long long* er = reinterpret_cast<long long*>(w + o_er);
  int* lsr = reinterpret_cast<int*>(w + o_ls);
  int* br = reinterpret_cast<int*>(w + o_br);
  float* be = reinterpret_cast<float*>(w + o_be);
  float* bg = reinterpret_cast<float*>(w + o_bg);
  float* bx = reinterpret_cast<float*>(w + o_bx);

  LaunchTimer timer(s);
  const LigDev& L = lig->dev;
  const RecDev& R = rec->dev;
  hipError_t e = hipMemsetAsync(er, 0, (size_t)runs * 8, s);
  if (e == hipSuccess)
    e = timer.run(MD_K_INIT_POPULATION, [&] { return launch_init_population(L, R, P, ga, ea, ev, s); });
  if (e == hipSuccess) e = timer.run(MD_K_SUM_EVALS, [&] { return launch_sum_evals(P, ev, er, s); });
  for (int g = 1; g <= gens && e == hipSuccess; ++g) {
    e = timer.run(MD_K_GENERATION, [&] { return launch_generation(L, R, P, g, ga, ea, gb, eb, ev, s); });
    if (e == hipSuccess && n_ls > 0)
      e = timer.run(MD_K_LS_PICK, [&] { return launch_ls_pick(P, g, lsr, s); });
    if (e == hipSuccess && n_ls > 0)
      e = timer.run(MD_K_LOCAL_SEARCH, [&] {
        return launch_local_search(L, R, runs * n_ls, lsr, gb, gb, eb, ev, P.ls_iters, P.rho, P.eps,
                                   nullptr, s);
      });
    if (e == hipSuccess) e = timer.run(MD_K_SUM_EVALS, [&] { return launch_sum_evals(P, ev, er, s); });
    std::swap(ga, gb);
    std::swap(ea, eb);
  }
  if (e == hipSuccess)
    e = timer.run(MD_K_BEST_OF_RUNS, [&] { return launch_best_of_runs(P, ga, ea, br, be, bg, s); });
  if (e == hipSuccess && out->best_xyz) e = launch_pose(lig->dev, runs, bg, bx, s);
  std::vector<float> h_be(runs), h_bg((size_t)runs * G), h_bx(out->best_xyz ? (size_t)runs * N * 3 : 0);
  std::vector<long long> h_er(runs);
  if (e == hipSuccess) e = hipMemcpyAsync(h_be.data(), be, runs * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h_bg.data(), bg, (size_t)runs * G * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h_er.data(), er, (size_t)runs * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && out->best_xyz)
    e = hipMemcpyAsync(h_bx.data(), bx, h_bx.size() * 4, hipMemcpyDeviceToHost, s);
  hipError_t ef = hipFreeAsync(w, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  timer.collect(e == hipSuccess);
  if (e != hipSuccess) return hip_fail(e, "md_dock");

  std::vector<int> order(runs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h_be[a] < h_be[b]; });
  for (int k = 0; k < runs; ++k) {
    const int r = order[k];
    out->best_energy[k] = h_be[r];
    std::memcpy(out->best_genes + (size_t)k * out->n_genes, h_bg.data() + (size_t)r * G, G * 4);
    if (out->best_xyz)
      std::memcpy(out->best_xyz + (size_t)k * out->n_atoms * 3, h_bx.data() + (size_t)r * N * 3, (size_t)N * 12);
    if (out->run_index) out->run_index[k] = r;
    if (out->evals) out->evals[k] = h_er[r];
    if (out->generations) out->generations[k] = gens;
  }
  return MD_OK;
}

}  // extern "C"
