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

// Generations per captured graph of md_dock_batch: fewer joins of the size classes' branches.
constexpr int kBatchGraphGenerations = 4;

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

}  // namespace

namespace mdock {

// One device allocation per ligand holding every constant the kernels read; *L gets views into it.
hipError_t upload_ligand(const LigHost& h, void** d_buf, LigDev* L) {
  const size_t N = h.n_atoms, T = h.n_tors, S = h.pair_ij.size() + kWave;   // S: scheduled slots + a pad row
  size_t off = 0;
  const size_t o_p0q = off; off = align16(off + N * sizeof(float4));
  const size_t o_type = off; off = align16(off + N * sizeof(int));
  const size_t o_mask = off; off = align16(off + N * sizeof(uint32_t));
  const size_t o_axis = off; off = align16(off + T * sizeof(float4));
  const size_t o_piv = off; off = align16(off + T * sizeof(float4));
  const size_t o_ab = off; off = align16(off + T * sizeof(int2));
  const size_t o_gene = off; off = align16(off + T * sizeof(int));
  const size_t o_gtor = off; off = align16(off + T * sizeof(int));
  const size_t o_ij = off; off = align16(off + S * sizeof(uint32_t));
  const size_t o_coef = off; off = align16(off + S * sizeof(float4));
  std::vector<char> buf(std::max<size_t>(off, 16), 0);
  auto put = [&](size_t o, const void* p, size_t n) { if (n) std::memcpy(buf.data() + o, p, n); };
  put(o_p0q, h.atom_p0q.data(), N * sizeof(float4));
  put(o_type, h.atom_type.data(), N * sizeof(int));
  put(o_mask, h.atom_mask.data(), N * sizeof(uint32_t));
  put(o_axis, h.tor_axis.data(), T * sizeof(float4));
  put(o_piv, h.tor_pivot.data(), T * sizeof(float4));
  put(o_ab, h.tor_ab.data(), T * sizeof(int2));
  put(o_gene, h.tor_gene.data(), T * sizeof(int));
  put(o_gtor, h.gene_tor.data(), T * sizeof(int));
  // device slots: byte offsets of the two atoms' entries; then a padding row of empty slots
  std::vector<uint32_t> ij(S, (uint32_t)(4 * N) | ((uint32_t)(4 * N) << 16));
  for (size_t k = 0; k < h.pair_ij.size(); ++k)
    ij[k] = 4u * (h.pair_ij[k] & 0xffu) | ((4u * ((h.pair_ij[k] >> 8) & 0xffu)) << 16);
  put(o_ij, ij.data(), S * sizeof(uint32_t));
  // the second coefficient of an H-bond pair is stored negated (its 12-10 marker)
  std::vector<float4> coef(h.pair_coef);
  for (size_t k = 0; k < coef.size(); ++k)
    if ((h.pair_ij[k] >> 16) & 1u) coef[k].y = -coef[k].y;
  put(o_coef, coef.data(), coef.size() * sizeof(float4));
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, buf.size());
  if (e == hipSuccess) e = hipMemcpy(d, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (d) (void)hipFree(d);
    return e;
  }
  char* b = static_cast<char*>(d);
  LigDev& l = *L;
  l.n_atoms = (int)N;
  l.n_tors = (int)T;
  l.n_pairs = h.n_pairs;
  l.n_genes = h.n_genes;
  l.atom_p0q = reinterpret_cast<const float4*>(b + o_p0q);
  l.atom_type = reinterpret_cast<const int*>(b + o_type);
  l.atom_mask = reinterpret_cast<const uint32_t*>(b + o_mask);
  l.tor_axis = reinterpret_cast<const float4*>(b + o_axis);
  l.tor_pivot = reinterpret_cast<const float4*>(b + o_piv);
  l.tor_ab = reinterpret_cast<const int2*>(b + o_ab);
  l.tor_gene = reinterpret_cast<const int*>(b + o_gene);
  l.gene_tor = reinterpret_cast<const int*>(b + o_gtor);
  l.pair_ij = reinterpret_cast<const uint32_t*>(b + o_ij);
  l.pair_coef = reinterpret_cast<const float4*>(b + o_coef);
  l.n_rows = h.n_rows;
  l.mix_rows = h.mix_rows;
  l.pl_rows = h.pl_rows;
  l.group_lanes = h.group_lanes;
  l.n_copies = h.n_copies;
  l.wpb = h.wpb;
  l.wpp = h.wpp;
  l.lds_bytes = h.lds_bytes;
  *d_buf = d;
  return hipSuccess;
}

md_status api_fail(md_status st, const std::string& msg) { return fail(st, msg); }
md_status api_hip_fail(hipError_t e, const std::string& what) { return hip_fail(e, what.c_str()); }

}  // namespace mdock

namespace {

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
  const long long elem_bytes = stored == MD_MAP_FP32 ? 4 : 2;
  if (nodes > ((1ll << 31) - 1) / (kCellValues * elem_bytes))
    return fail(MD_ERANGE, "md_receptor_create: grid too large (the stored cell records must stay below 2 GiB)");
  const long long count = nodes * kMaps;
  for (long long i = 0; i < count; ++i)
    if (!std::isfinite(maps[i])) return fail(MD_EINVAL, "md_receptor_create: non-finite map value");
  if (stored == MD_MAP_FP16)
    for (long long i = 0; i < count; ++i)
      if (std::fabs(maps[i]) > 65504.f) return fail(MD_ERANGE, "md_receptor_create: map value outside FP16 range");

  // device layout: one record per cell, named by its lowest node (x fastest), holding the
  // cell's eight corner values (corner bit 0 +x, bit 1 +y, bit 2 +z): the type maps' records
  // [7][cells][8], then the electrostatic and desolvation maps' [cells][8][2] (every atom reads
  // both at the same corners).  An atom's 24 corner values are then three aligned 32- or
  // 64-byte runs, whatever its cell; corners past the last node (records of the last layer,
  // which no inside atom reads) hold zero.
  const size_t elem = stored == MD_MAP_FP32 ? 4 : 2;
  const long long dcount = nodes * kCellValues;
  std::vector<float> f32;
  std::vector<uint16_t> f16;
  try {
    if (stored == MD_MAP_FP32)
      f32.assign((size_t)dcount, 0.f);
    else
      f16.assign((size_t)dcount, 0);
  } catch (const std::bad_alloc&) {
    return fail(MD_ENOMEM, "md_receptor_create: out of host memory for the cell records");
  }
  auto put = [&](long long k, float v) {
    if (stored == MD_MAP_FP32)
      f32[(size_t)k] = v;
    else
      f16[(size_t)k] = stored == MD_MAP_FP16 ? f32_to_f16_rne(v) : f32_to_bf16_rne(v);
  };
  const long long ed = (long long)kTypes * nodes * 8;
  for (long long z = 0; z < d->nz; ++z)
    for (long long y = 0; y < d->ny; ++y)
      for (long long x = 0; x < d->nx; ++x) {
        const long long cell = (z * d->ny + y) * d->nx + x;
        for (int c = 0; c < 8; ++c) {
          const long long cx = x + (c & 1), cy = y + ((c >> 1) & 1), cz = z + (c >> 2);
          if (cx >= d->nx || cy >= d->ny || cz >= d->nz) continue;
          const long long node = (cz * d->ny + cy) * d->nx + cx;
          for (int t = 0; t < kTypes; ++t) put(((long long)t * nodes + cell) * 8 + c, maps[t * nodes + node]);
          put(ed + cell * 16 + 2 * c, maps[kTypes * nodes + node]);
          put(ed + cell * 16 + 2 * c + 1, maps[(kTypes + 1) * nodes + node]);
        }
      }
  const void* src = stored == MD_MAP_FP32 ? static_cast<const void*>(f32.data()) : static_cast<const void*>(f16.data());
  md_receptor* r = new (std::nothrow) md_receptor();
  if (!r) return fail(MD_ENOMEM, "md_receptor_create: out of host memory");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&r->device);
  if (e == hipSuccess) e = hipMalloc(&r->d_maps, dcount * elem);
  if (e == hipSuccess) e = hipMemcpyAsync(r->d_maps, src, dcount * elem, hipMemcpyHostToDevice, s);
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
  R.map_bytes = (unsigned)(dcount * elem);
  R.gx_max = (float)(d->nx - 1);
  R.gy_max = (float)(d->ny - 1);
  R.gz_max = (float)(d->nz - 1);
  R.hx = R.ox + R.gx_max * R.h;
  R.hy = R.oy + R.gy_max * R.h;
  R.hz = R.oz + R.gz_max * R.h;
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
  // the default plan, whatever was tuned earlier in the process: a tuned plan changes the order
  // of floating-point sums, so applying it is the caller's choice (md_ligand_autotune reads the
  // tune table), never a side effect of creation
  hipError_t e = hipGetDevice(&l->device);
  if (e == hipSuccess) e = enable_large_lds();
  if (e == hipSuccess) e = upload_ligand(l->host, &l->d_buf, &l->dev);
  if (e != hipSuccess) {
    delete l;
    return hip_fail(e, "md_ligand_create");
  }
  *out = l;
  return MD_OK;
}

md_status md_ligand_destroy(md_ligand* l) {
  if (!l) return MD_OK;
  if (l->holds.load() > 0) return fail(MD_EBUSY, "md_ligand_destroy: a server request still uses the ligand");
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

md_status md_set_graphs(int on) {
  set_use_graphs(on != 0);
  return MD_OK;
}

int md_graphs_enabled(void) { return use_graphs() ? 1 : 0; }

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

namespace {
md_status local_search_common(const char* who, const md_receptor* rec, const md_ligand* lig, int n,
                              const float* genes_in, float* genes_out, float* energy_out, int n_iters, float rho,
                              float eps, float* trace, float* trace_x, float* trace_g, void* hip_stream) {
  const std::string w(who);
  if (!rec || !lig) return fail(MD_EINVAL, w + ": null handle");
  if (n < 0) return fail(MD_EINVAL, w + ": n < 0");
  if (n_iters < 1) return fail(MD_EINVAL, w + ": n_iters must be >= 1");
  if (!(rho >= 0.f && rho < 1.f) || !(eps > 0.f) || !std::isfinite(eps))
    return fail(MD_EINVAL, w + ": rho must be in [0,1) and eps > 0");
  if (n == 0) return MD_OK;
  if (!genes_in || !genes_out || !energy_out) return fail(MD_EINVAL, w + ": null buffer");
  MD_HIP(launch_local_search(lig->dev, rec->dev, n, genes_in, genes_out, energy_out, n_iters, rho, eps, trace,
                             trace_x, trace_g, static_cast<hipStream_t>(hip_stream)),
         (w + " launch").c_str());
  return MD_OK;
}
}  // namespace

md_status md_local_search(const md_receptor* rec, const md_ligand* lig, int n, const float* genes_in,
                          float* genes_out, float* energy_out, int n_iters, float rho, float eps,
                          float* trace, void* hip_stream) {
  return local_search_common("md_local_search", rec, lig, n, genes_in, genes_out, energy_out, n_iters, rho, eps,
                             trace, nullptr, nullptr, hip_stream);
}

md_status md_local_search_traced(const md_receptor* rec, const md_ligand* lig, int n, const float* genes_in,
                                 float* genes_out, float* energy_out, int n_iters, float rho, float eps,
                                 float* trace, float* trace_genes, float* trace_grad, void* hip_stream) {
  return local_search_common("md_local_search_traced", rec, lig, n, genes_in, genes_out, energy_out, n_iters, rho,
                             eps, trace, trace_genes, trace_grad, hip_stream);
}

md_status md_local_search_sw(const md_receptor* rec, const md_ligand* lig, int n, const float* genes_in,
                             float* genes_out, float* energy_out, int n_evals, unsigned long long seed,
                             float* trace, void* hip_stream) {
  if (!rec || !lig) return fail(MD_EINVAL, "md_local_search_sw: null handle");
  if (n < 0) return fail(MD_EINVAL, "md_local_search_sw: n < 0");
  if (n_evals < 1) return fail(MD_EINVAL, "md_local_search_sw: n_evals must be >= 1");
  if (n_evals > (1 << 24)) return fail(MD_ERANGE, "md_local_search_sw: n_evals must be <= 2^24");
  if (n == 0) return MD_OK;
  if (!genes_in || !genes_out || !energy_out) return fail(MD_EINVAL, "md_local_search_sw: null buffer");
  MD_HIP(launch_solis_wets(lig->dev, rec->dev, n, genes_in, genes_out, energy_out, n_evals, seed, trace,
                           static_cast<hipStream_t>(hip_stream)),
         "md_local_search_sw launch");
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

}  // extern "C"

namespace {

std::string check_params(const md_dock_params* p) {
  if (p->n_runs < 1 || p->pop_size < 2) return "need n_runs >= 1 and pop_size >= 2";
  if (p->pop_size > 1024) return "pop_size must be <= 1024";
  if ((long long)p->n_runs * p->pop_size > (1ll << 26)) return "n_runs * pop_size too large";
  if (p->elitism != 0 && p->elitism != 1) return "elitism must be 0 or 1";
  if (p->max_generations < 0 || p->max_evals_per_run < 0) return "negative budget";
  if (!(p->ls_rate >= 0.f && p->ls_rate <= 1.f)) return "ls_rate must be in [0,1]";
  if (n_local_search(p) > 0 && p->ls_iters < 1) return "ls_iters must be >= 1";
  if (p->ls_method != MD_LS_ADADELTA && p->ls_method != MD_LS_SOLIS_WETS) return "unknown ls_method";
  if (p->ls_method == MD_LS_SOLIS_WETS && p->ls_iters > (1 << 24)) return "Solis-Wets ls_iters must be <= 2^24";
  if (!(p->rho >= 0.f && p->rho < 1.f) || !(p->eps > 0.f)) return "bad rho/eps";
  const float rates[3] = {p->crossover_rate, p->mutation_rate, p->tournament_rate};
  for (float r : rates)
    if (!(r >= 0.f && r <= 1.f)) return "rates must be in [0,1]";
  if (!std::isfinite(p->mut_trans) || !std::isfinite(p->mut_rot) || !std::isfinite(p->mut_tors))
    return "non-finite mutation size";
  return std::string();
}

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align16(off + bytes);
    return o;
  }
};

}  // namespace

namespace mdock {
md_status server_fail(md_status st, const std::string& msg) { return fail(st, msg); }
int n_local_search_of(const md_dock_params* p) { return n_local_search(p); }
std::string check_dock_params(const md_dock_params* p) { return check_params(p); }
}  // namespace mdock

extern "C" {

md_status md_dock_batch(const md_receptor* rec, int n_jobs, const md_dock_job* jobs, void* hip_stream) {
  if (!rec || n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(MD_EINVAL, "md_dock_batch: null argument");
  if (n_jobs == 0) return MD_OK;
  if (n_jobs > (1 << 20)) return fail(MD_ERANGE, "md_dock_batch: too many jobs");
  for (int j = 0; j < n_jobs; ++j) {
    const md_dock_job& jb = jobs[j];
    if (!jb.ligand || !jb.result) return fail(MD_EINVAL, "md_dock_batch: job " + std::to_string(j) + ": null ligand or result");
    const std::string e = check_params(&jb.params);
    if (!e.empty()) {
      const bool range = e.find("<=") != std::string::npos || e.find("too large") != std::string::npos;
      return fail(range ? MD_ERANGE : MD_EINVAL, "md_dock_batch: job " + std::to_string(j) + ": " + e);
    }
    const md_dock_result* out = jb.result;
    const int G = jb.ligand->dev.n_genes, N = jb.ligand->dev.n_atoms;
    if (out->n_runs < jb.params.n_runs || out->n_genes < G || !out->best_energy || !out->best_genes)
      return fail(MD_EINVAL, "md_dock_batch: job " + std::to_string(j) + ": result buffers too small or null");
    if (out->best_xyz && out->n_atoms < N)
      return fail(MD_EINVAL, "md_dock_batch: job " + std::to_string(j) + ": best_xyz capacity too small");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);

  // workspace: job table, block tables, per-job populations, then one results region
  std::vector<JobDev> table(n_jobs);
  std::vector<SchedJob> sched_jobs(n_jobs);
  int max_planned = 0;
  Carve cv;
  const size_t o_table = cv.take(sizeof(JobDev) * n_jobs);
  struct Offs { size_t ga, gb, ea, eb, ev, lsr, br; size_t be, bg, er, bx; };
  std::vector<Offs> offs(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    const md_dock_params& p = jobs[j].params;
    const LigDev& L = jobs[j].ligand->dev;
    const size_t rows = (size_t)p.n_runs * p.pop_size;
    const int n_ls = n_local_search(&p);
    Offs& o = offs[j];
    o.ga = cv.take(rows * L.n_genes * 4);
    o.gb = cv.take(rows * L.n_genes * 4);
    o.ea = cv.take(rows * 4);
    o.eb = cv.take(rows * 4);
    o.ev = cv.take(rows * 4);
    o.lsr = cv.take((size_t)p.n_runs * std::max(n_ls, 1) * 4);
    o.br = cv.take((size_t)p.n_runs * 4);
    sched_jobs[j] = SchedJob{j, &jobs[j].ligand->dev, p.n_runs, p.pop_size, n_ls, p.ls_iters, p.ls_method};
    max_planned = std::max(max_planned, md_dock_planned_generations(&p));
  }
  GenSchedule sched;
  build_schedule(sched_jobs, sched, 0, kBatchGraphGenerations);
  const size_t o_blocks = cv.take(sizeof(int2) * std::max<size_t>(sched.blocks.size(), 1));
  const size_t o_results = cv.off;
  for (int j = 0; j < n_jobs; ++j) {
    const md_dock_params& p = jobs[j].params;
    const LigDev& L = jobs[j].ligand->dev;
    Offs& o = offs[j];
    o.be = cv.take((size_t)p.n_runs * 4);
    o.bg = cv.take((size_t)p.n_runs * L.n_genes * 4);
    o.er = cv.take((size_t)p.n_runs * 8);
    o.bx = jobs[j].result->best_xyz ? cv.take((size_t)p.n_runs * L.n_atoms * 12) : 0;
  }
  const size_t results_bytes = cv.off - o_results;

  char* w = nullptr;
  MD_HIP(hipMallocAsync(reinterpret_cast<void**>(&w), cv.off, s), "md_dock workspace");
  for (int j = 0; j < n_jobs; ++j) {
    const md_dock_params& p = jobs[j].params;
    const Offs& o = offs[j];
    JobDev& J = table[j];
    J.L = jobs[j].ligand->dev;
    GaDev& P = J.P;
    P.n_runs = p.n_runs;
    P.pop_size = p.pop_size;
    P.n_genes = J.L.n_genes;
    P.n_ls = n_local_search(&p);
    P.ls_iters = p.ls_iters;
    P.ls_method = p.ls_method;
    P.elitism = p.elitism;
    P.rho = p.rho;
    P.eps = p.eps;
    P.crossover_rate = p.crossover_rate;
    P.mutation_rate = p.mutation_rate;
    P.tournament_rate = p.tournament_rate;
    P.mut_trans = p.mut_trans;
    P.mut_rot = p.mut_rot;
    P.mut_tors = p.mut_tors;
    P.seed = p.seed;
    J.genes[0] = reinterpret_cast<float*>(w + o.ga);
    J.genes[1] = reinterpret_cast<float*>(w + o.gb);
    J.energy[0] = reinterpret_cast<float*>(w + o.ea);
    J.energy[1] = reinterpret_cast<float*>(w + o.eb);
    J.evals = reinterpret_cast<int*>(w + o.ev);
    J.evals_of_runs = reinterpret_cast<long long*>(w + o.er);
    J.ls_rows = reinterpret_cast<int*>(w + o.lsr);
    J.best_row = reinterpret_cast<int*>(w + o.br);
    J.best_energy = reinterpret_cast<float*>(w + o.be);
    J.best_genes = reinterpret_cast<float*>(w + o.bg);
    J.best_xyz = jobs[j].result->best_xyz ? reinterpret_cast<float*>(w + o.bx) : nullptr;
    J.gen = 0;
    J.cur = 0;
    J.planned = md_dock_planned_generations(&p);
    J.state = kJobInit;
  }
  JobDev* d_table = reinterpret_cast<JobDev*>(w + o_table);
  const int2* d_blocks = reinterpret_cast<const int2*>(w + o_blocks);
  const RecDev& R = rec->dev;

  // Initial populations, then the generations: when profiling, phase by phase (each phase's
  // class launches concurrent, the phase timed) or, without graphs, one launch at a time; else
  // one captured generation replayed max_planned times (jobs that finish early skip the rest on
  // the device).
  LaunchTimer timer(s);
  const LaunchHook hook = [&](int kind, const std::function<hipError_t()>& f) { return timer.run(kind, f); };
  hipError_t e = hipMemcpyAsync(d_table, table.data(), sizeof(JobDev) * n_jobs, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !sched.blocks.empty())
    e = hipMemcpyAsync(w + o_blocks, sched.blocks.data(), sizeof(int2) * sched.blocks.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_init_phase(sched, d_table, d_blocks, R, s, &hook);
  if (e == hipSuccess) e = timer.run(MD_K_SUM_EVALS, [&] { return launch_ga_advance(d_table, n_jobs, s); });
  if (g_prof.on && use_graphs() && max_planned >= 2) {
    // timed: each phase's launches concurrent over the classes, as the captured generation runs
    // them, and the phase bracketed by the timer
    GenGraph branches;
    for (int g = 1; g <= max_planned && e == hipSuccess; ++g)
      e = branches.launch_phased(sched, d_table, d_blocks, R, s, &hook);
    // the branch streams are destroyed with `branches`: finish their work first
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else if (g_prof.on || !use_graphs() || max_planned < 2) {
    for (int g = 1; g <= max_planned && e == hipSuccess; ++g)
      e = launch_generation_phase(sched, d_table, d_blocks, R, s, &hook);
  } else {
    // each replay runs kBatchGraphGenerations generations of every class (the classes as
    // parallel branches); generations past a job's plan are skipped on the device
    GenGraph graph;
    if (e == hipSuccess) e = graph.capture(sched, d_table, d_blocks, R);
    const int replays = (max_planned + kBatchGraphGenerations - 1) / kBatchGraphGenerations;
    for (int g = 0; g < replays && e == hipSuccess; ++g) e = graph.launch(s);
    // the graph's launches read the workspace: finish them before the graph is destroyed
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  // the epilogue that finished each job wrote its best genes, energies and poses
  std::vector<char> host(results_bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), w + o_results, results_bytes, hipMemcpyDeviceToHost, s);
  hipError_t ef = hipFreeAsync(w, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  timer.collect(e == hipSuccess);
  if (e != hipSuccess) return hip_fail(e, "md_dock");

  for (int j = 0; j < n_jobs; ++j) {
    const md_dock_params& p = jobs[j].params;
    md_dock_result* out = jobs[j].result;
    const int runs = p.n_runs, G = table[j].L.n_genes, N = table[j].L.n_atoms;
    const float* be = reinterpret_cast<const float*>(host.data() + (offs[j].be - o_results));
    const float* bg = reinterpret_cast<const float*>(host.data() + (offs[j].bg - o_results));
    const long long* er = reinterpret_cast<const long long*>(host.data() + (offs[j].er - o_results));
    const float* bx = out->best_xyz ? reinterpret_cast<const float*>(host.data() + (offs[j].bx - o_results)) : nullptr;
    std::vector<int> order(runs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return be[a] < be[b]; });
    for (int k = 0; k < runs; ++k) {
      const int r = order[k];
      out->best_energy[k] = be[r];
      std::memcpy(out->best_genes + (size_t)k * out->n_genes, bg + (size_t)r * G, (size_t)G * 4);
      if (out->best_xyz) std::memcpy(out->best_xyz + (size_t)k * out->n_atoms * 3, bx + (size_t)r * N * 3, (size_t)N * 12);
      if (out->run_index) out->run_index[k] = r;
      if (out->evals) out->evals[k] = er[r];
      if (out->generations) out->generations[k] = table[j].planned;
    }
  }
  return MD_OK;
}

md_status md_dock(const md_receptor* rec, const md_ligand* lig, const md_dock_params* p,
                  md_dock_result* out, void* hip_stream) {
  if (!rec || !lig || !p || !out) return fail(MD_EINVAL, "md_dock: null argument");
  md_dock_job job;
  job.ligand = lig;
  job.params = *p;
  job.result = out;
  return md_dock_batch(rec, 1, &job, hip_stream);
}

}  // extern "C"
