// gfx950 kernels of libmdock: pose, energy and genotype gradient, ADADELTA and Solis-Wets
// local searches, GA generation, evaluation accounting and best-of-runs.
//
// Mapping: one 64-lane wavefront owns one pose (genotype).  Lanes hold atoms (atom l and,
// for ligands above 64 atoms, l + 64), then stride over the intramolecular pair list; the
// per-pose energy and the genotype gradient are wavefront reductions.  Waves of a block are
// independent (no block barriers), so a block can hold poses of different work.  A plan may
// instead let the 2 or 4 waves of a block share one local-search pose (eval_pose_shared):
// they split the posing, the pair rows and the torsion gradients and meet in LDS at block
// barriers, for searches too few to fill the device.
//
// Paper passages: the energy kernel's phases -- per-atom positions, rotations in a fixed
// order, per-atom energy sum (Section "Approach 1", listing of decomposed target
// functions) -- and the per-run evaluation sum (Section "Removing architecture-specific
// code", sum_evals listings).  The method (grid receptor, ligand self-interactions,
// Lamarckian GA with a local search on a random sample, several runs, best over runs) is
// from Background, "Design and Structure of MiniMDock".
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <set>

#include "internal.h"

namespace mdock {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;

// ------------------------------------------------------------------ wave utilities
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Makes this wave's LDS writes visible to its other lanes and keeps the compiler from
// moving LDS accesses across the point (a wavefront executes its LDS operations in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Wavefront sum through DPP lane moves: quad swaps, half-row and row mirrors, then the row
// broadcasts of lanes 15 and 31; lane 63 ends with the total, which is returned to every lane
// (a wave-uniform value).  The addition order is fixed, so the result is deterministic.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp<0x141, 0xf>(v);   // row_half_mirror
  v += dpp<0x140, 0xf>(v);   // row_mirror
  v += dpp<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return readlane(v, 63);
}

// Wavefront sum by the tree the gradient path's reduce-scatter gives the energy (rigid_gradient
// with WITH_E): each lane adds its partner 32 lanes away, then the partner row, then the row is
// summed by DPP; so the energy-only and the gradient evaluations agree bitwise.
__device__ __forceinline__ float wave_sum_rs(float v) {
  const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const float h = __uint_as_float(s[0]) + __uint_as_float(s[1]);
  const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(h), __float_as_uint(h), false, false);
  float r = __uint_as_float(t[0]) + __uint_as_float(t[1]);
  r += dpp<0xb1, 0xf>(r);    // quad_perm [1,0,3,2]
  r += dpp<0x4e, 0xf>(r);    // quad_perm [2,3,0,1]
  r += dpp<0x141, 0xf>(r);   // row_half_mirror
  r += dpp<0x140, 0xf>(r);   // row_mirror
  return readlane(r, 16);
}

// ------------------------------------------------------------------ counter-based RNG
// SplitMix64 (Steele, Lea, Flood 2014) folded over the draw's coordinates.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum : uint32_t { kPInit = 1, kPTournament = 2, kPCrossover = 3, kPMutation = 4, kPLsPick = 5, kPLsSw = 6 };

__device__ __forceinline__ uint32_t draw_u24(uint64_t seed, uint32_t run, uint32_t gen,
                                             uint32_t indiv, uint32_t purpose, uint32_t index) {
  uint64_t h = seed;
  h = splitmix64(h ^ run);
  h = splitmix64(h ^ gen);
  h = splitmix64(h ^ indiv);
  h = splitmix64(h ^ purpose);
  h = splitmix64(h ^ index);
  return (uint32_t)(h >> 40);
}

// The hash state after the first five coordinates; draw_from(prefix, index) then equals
// draw_u24(seed, run, gen, indiv, purpose, index) at one mixing round per draw.
__device__ __forceinline__ uint64_t draw_prefix(uint64_t seed, uint32_t run, uint32_t gen, uint32_t indiv,
                                                uint32_t purpose) {
  uint64_t h = seed;
  h = splitmix64(h ^ run);
  h = splitmix64(h ^ gen);
  h = splitmix64(h ^ indiv);
  return splitmix64(h ^ purpose);
}

__device__ __forceinline__ uint32_t draw_from(uint64_t prefix, uint32_t index) {
  return (uint32_t)(splitmix64(prefix ^ index) >> 40);
}

__device__ __forceinline__ float draw_uniform(uint64_t seed, uint32_t run, uint32_t gen,
                                              uint32_t indiv, uint32_t purpose, uint32_t index) {
  return (float)draw_u24(seed, run, gen, indiv, purpose, index) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ int draw_int(int n, uint64_t seed, uint32_t run, uint32_t gen,
                                        uint32_t indiv, uint32_t purpose, uint32_t index) {
  return (int)(((uint64_t)draw_u24(seed, run, gen, indiv, purpose, index) * (uint64_t)n) >> 24);
}

__device__ __forceinline__ float wrap_angle(float th) {
  return th - kTwoPi * ceilf((th - kPi) * (1.0f / kTwoPi));
}

// ------------------------------------------------------------------ LDS layout
// Dynamic LDS of a block (sizes from the ligand's plan): the staged pair rows, shared by the
// block's waves; then per wave the posed coordinates and the force-array copies, one per lane
// group of the pair schedule; then, when the block's waves share one pose, the share sets
// (partial forces and energies, see eval_pose).
struct BlockLds {
  const float4* pair_coef;   // [(pl_rows + 1)*64]
  const uint32_t* pair_ij;   // [(pl_rows + 1)*64]
  float* x;                  // this wave: posed x, y, z as [3][64A + 1]
  float* f;                  // this wave: [n_copies] blocks of intramolecular forces [3][64A + 1]
  float* fg;                 // this lane's group copy
  float4* tor;               // this wave: [3*roundup4(n_tors)] torsion table (see eval_pose)
  float4* share;             // waves sharing a pose: the pose's coordinates, then two sets of
                             // [W + 1][n_atoms + 1] + [W] (see eval_pose_shared)
};

// x, y, z of entry i of a coordinate or force array of pitch 64A + 1
template <int A>
__device__ __forceinline__ float3 load3(const float* a, int i) {
  constexpr int P = kWave * A + 1;
  return make_float3(a[i], a[P + i], a[2 * P + i]);
}
template <int A>
__device__ __forceinline__ void store3(float* a, int i, float x, float y, float z) {
  constexpr int P = kWave * A + 1;
  a[i] = x;
  a[P + i] = y;
  a[2 * P + i] = z;
}

// Which of the waves sharing a pose this one is, and which share set its next evaluation uses
// (sets alternate, so one barrier per evaluation suffices: a wave can rewrite a set only after
// every wave has passed the next evaluation's barrier, i.e. has finished reading it).
struct PoseShare {
  int w;
  int par;
};

extern __shared__ __align__(16) unsigned char g_lds[];

// All threads of the block stage the shared part and clear their wave's coordinate and force
// arrays, then synchronise.  Must be reached by every wave of the block before any leaves.
template <int A>
__device__ __forceinline__ BlockLds stage_block(const LigDev& L) {
  BlockLds b;
  unsigned char* cur = g_lds;
  const int ns = lds_staged_rows(L.pl_rows) * kWave;
  float4* pc = reinterpret_cast<float4*>(cur);
  uint32_t* pij = reinterpret_cast<uint32_t*>(cur + (size_t)ns * 16);
  cur += lds_pairs_bytes(L.pl_rows);
  for (int p = threadIdx.x; p < ns; p += blockDim.x) {
    pc[p] = L.pair_coef[p];
    pij[p] = L.pair_ij[p];
  }
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const size_t wave_bytes = lds_wave_bytes(L.n_atoms, L.n_copies, A, L.n_tors);
  b.share = reinterpret_cast<float4*>(cur + (size_t)L.wpb * wave_bytes);
  cur += (size_t)w * wave_bytes;
  b.pair_coef = pc;
  b.pair_ij = pij;
  const size_t cb = lds_coord_bytes(A);
  b.x = reinterpret_cast<float*>(cur);
  cur += cb;
  b.f = reinterpret_cast<float*>(cur);
  cur += cb * L.n_copies;
  b.tor = reinterpret_cast<float4*>(cur);
  if (lane == 0) store3<A>(b.x, kWave * A, 0.f, 0.f, 0.f);
  if (L.wpp > 1 && threadIdx.x == 0)   // spare entry of the shared pose's coordinates
    store3<A>(reinterpret_cast<float*>(b.share), kWave * A, 0.f, 0.f, 0.f);
  const int nf = (int)(L.n_copies * cb / 4);
  for (int k = lane; k < nf; k += kWave) b.f[k] = 0.f;
  const int g = min(lane / L.group_lanes, max(L.n_copies - 1, 0));
  b.fg = b.f + g * (cb / 4);
  __syncthreads();
  return b;
}

// Per-lane ligand constants for A atoms per lane (atom lane + 64*a) and, in lanes k < T, the
// constants of torsion k (reference axis and pivot, its two atoms, its gene index).  Loops over
// torsions fetch them with readlane, so the inner loops touch no memory.
template <int A>
struct AtomRegs {
  float px[A], py[A], pz[A], q[A];
  uint32_t tofs[A];          // record offset of the atom's type map (type * cells)
  uint32_t mask[A];
  bool valid[A];
  int gene_of_tor;
  int tor_of_gene;           // lanes 7 .. G-1: internal torsion of gene `lane`
  float tux, tuy, tuz, tpx, tpy, tpz;
  int ta, tb;
};

template <int A>
__device__ __forceinline__ void load_ligand(const LigDev& L, AtomRegs<A>& at, long long map_stride = 0) {
  const int lane = lane_id();
#pragma unroll
  for (int a = 0; a < A; ++a) {
    int i = lane + kWave * a;
    at.valid[a] = i < L.n_atoms;
    float4 p = at.valid[a] ? L.atom_p0q[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    at.px[a] = p.x;
    at.py[a] = p.y;
    at.pz[a] = p.z;
    at.q[a] = p.w;
    at.tofs[a] = at.valid[a] ? (uint32_t)L.atom_type[i] * (uint32_t)map_stride : 0u;
    at.mask[a] = at.valid[a] ? L.atom_mask[i] : 0u;
  }
  at.gene_of_tor = 0;
  at.tor_of_gene = (lane >= 7 && lane < L.n_genes) ? L.gene_tor[lane - 7] : 0;
  at.tux = at.tuy = at.tuz = at.tpx = at.tpy = at.tpz = 0.f;
  at.ta = at.tb = 0;
  if (lane < L.n_tors) {
    at.gene_of_tor = L.tor_gene[lane];
    const float4 u = L.tor_axis[lane], pv = L.tor_pivot[lane];
    const int2 ab = L.tor_ab[lane];
    at.tux = u.x;
    at.tuy = u.y;
    at.tuz = u.z;
    at.tpx = pv.x;
    at.tpy = pv.y;
    at.tpz = pv.z;
    at.ta = ab.x;
    at.tb = ab.y;
  }
}

// ------------------------------------------------------------------ grid term
// Trilinear interpolation of (type map + q * electrostatic + |q| * desolvation) and its
// derivative with respect to the atom position; out-of-grid penalty outside the box.
// Split in two so the corner loads are in flight while the pair term runs.
// The map allocation as a raw buffer resource: 32-bit byte offsets per lane, the wave-uniform
// parts of an address in the scalar offset, and reads past the allocation return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t map_rsrc(const RecDev& R) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(R.maps), 0, (int)R.map_bytes, 0x00020000);
}

// Two stored map values (FP16 or BF16 halves of a dword, low half first) as floats.
template <int PREC>
__device__ __forceinline__ void unpack2(uint32_t v, float& lo, float& hi) {
  if constexpr (PREC == 1) {
    lo = __half2float(__ushort_as_half((unsigned short)(v & 0xffffu)));
    hi = __half2float(__ushort_as_half((unsigned short)(v >> 16)));
  } else {
    lo = __uint_as_float(v << 16);
    hi = __uint_as_float(v & 0xffff0000u);
  }
}

struct GridFetch {
  float mt[8], me[8], md[8];   // corner values of the type, electrostatic and desolvation maps;
                               // corner bit0 = +x, bit1 = +y, bit2 = +z
  float fx, fy, fz;            // fractional position in the cell
  float ex, ey, ez;            // outside: offset from the box
  float q;
  bool inside;
};

// tofs: the record offset of the atom's type map (type * cells).  A cell's corner values are
// contiguous: 32 (FP32) or 16 bytes of the type map's record, 64 or 32 of the electrostatic and
// desolvation pairs, read with 16-byte loads whose record-internal steps, and the pairs' base,
// sit in the scalar offset.
template <int PREC>
__device__ __forceinline__ void grid_fetch(const RecDev& R, __amdgpu_buffer_rsrc_t rs, float x, float y, float z,
                                           uint32_t tofs, float q, bool valid, GridFetch& g) {
  constexpr uint32_t ES = PREC == 0 ? 4 : 2;   // bytes per stored value
  const float gx = (x - R.ox) * R.inv_h;
  const float gy = (y - R.oy) * R.inv_h;
  const float gz = (z - R.oz) * R.inv_h;
  g.inside = valid && gx >= 0.f && gy >= 0.f && gz >= 0.f && gx < R.gx_max && gy < R.gy_max && gz < R.gz_max;
  g.ex = x - fminf(fmaxf(x, R.ox), R.hx);
  g.ey = y - fminf(fmaxf(y, R.oy), R.hy);
  g.ez = z - fminf(fmaxf(z, R.oz), R.hz);
  g.fx = g.fy = g.fz = 0.f;
  g.q = q;
  // the corner values are read only where the atom is inside (grid_finish), so lanes outside
  // leave them unset
  if (g.inside) {
    const uint32_t ix = (uint32_t)gx, iy = (uint32_t)gy, iz = (uint32_t)gz;
    g.fx = __builtin_amdgcn_fractf(gx);   // gx - floor(gx), exact
    g.fy = __builtin_amdgcn_fractf(gy);
    g.fz = __builtin_amdgcn_fractf(gz);
    const uint32_t cell = (iz * (uint32_t)R.ny + iy) * (uint32_t)R.nx + ix;
    const uint32_t ot = (tofs + cell) * (8 * ES);                        // type-map record
    const uint32_t oe = cell * (16 * ES);                                // corner pairs
    const uint32_t se = (uint32_t)kTypes * (uint32_t)R.map_stride * (8 * ES);   // pairs' base
    if constexpr (PREC == 0) {
      const auto t0 = __builtin_amdgcn_raw_buffer_load_b128(rs, ot, 0u, 0);
      const auto t1 = __builtin_amdgcn_raw_buffer_load_b128(rs, ot, 16u, 0);
      uint32_t v[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, oe, se + 16u * k, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) v[4 * k + u] = w[u];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        g.mt[c] = __uint_as_float(t0[c]);
        g.mt[4 + c] = __uint_as_float(t1[c]);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        g.me[c] = __uint_as_float(v[2 * c]);
        g.md[c] = __uint_as_float(v[2 * c + 1]);
      }
    } else {
      const auto t = __builtin_amdgcn_raw_buffer_load_b128(rs, ot, 0u, 0);
      const auto w0 = __builtin_amdgcn_raw_buffer_load_b128(rs, oe, se, 0);
      const auto w1 = __builtin_amdgcn_raw_buffer_load_b128(rs, oe, se + 16u, 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        unpack2<PREC>(t[k], g.mt[2 * k], g.mt[2 * k + 1]);
        unpack2<PREC>(w0[k], g.me[k], g.md[k]);
        unpack2<PREC>(w1[k], g.me[4 + k], g.md[4 + k]);
      }
    }
  }
}

__device__ __forceinline__ float grid_finish(const RecDev& R, const GridFetch& g, bool valid, float& dx,
                                             float& dy, float& dz) {
  if (!valid) {
    dx = dy = dz = 0.f;
    return 0.f;
  }
  if (!g.inside) {
    dx = 2.f * kKout * g.ex;
    dy = 2.f * kKout * g.ey;
    dz = 2.f * kKout * g.ez;
    return kPout + kKout * (g.ex * g.ex + g.ey * g.ey + g.ez * g.ez);
  }
  float c[8];
  const float aq = fabsf(g.q);
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = g.mt[k] + g.q * g.me[k] + aq * g.md[k];
  // lerps a + f (b - a): the differences they form along x, y and z are the gradient's parts
  const float fx = g.fx, fy = g.fy, fz = g.fz;
  const float d00 = c[1] - c[0], d10 = c[3] - c[2], d01 = c[5] - c[4], d11 = c[7] - c[6];
  const float x00 = c[0] + fx * d00, x10 = c[2] + fx * d10, x01 = c[4] + fx * d01, x11 = c[6] + fx * d11;
  const float e0 = x10 - x00, e1 = x11 - x01;
  const float y0 = x00 + fy * e0, y1 = x01 + fy * e1;
  const float ez = y1 - y0;
  const float v = y0 + fz * ez;
  const float gx0 = d00 + fy * (d10 - d00), gx1 = d01 + fy * (d11 - d01);
  dx = (gx0 + fz * (gx1 - gx0)) * R.inv_h;
  dy = (e0 + fz * (e1 - e0)) * R.inv_h;
  dz = ez * R.inv_h;
  return v;
}

// ------------------------------------------------------------------ pair term
// Energy of one intramolecular pair at squared distance r2 and dE/dr / r (so that the force on
// i is that factor times (x_i - x_j)).  r is clamped to R_MIN with zero gradient below it.
// Four transcendentals: 1/r~ by rsq, the desolvation Gaussian and the dielectric exponential
// by exp2, and one reciprocal that serves both 1/eps and d eps/dr / eps:
//   eps = A + B/den = D/den with D = A den + B, so 1/eps = den^2 q and
//   (d eps/dr)/eps = B k lambda B e q, where q = 1/(den D).
// HB: 0 every pair 12-6, 2 per pair (12-10 where c.y < 0); |c.y| is the coefficient either way.
template <int HB>
__device__ __forceinline__ float pair_term(float r2, float4 c, float& f_over_r) {
  // No automatic contraction here: every fused multiply-add is written out, so the energy-only
  // and the gradient instantiations compute the energy with the same operations.
#pragma clang fp contract(off)
  const float rt2 = fmaxf(r2, kRmin * kRmin);
  const float ir = __builtin_amdgcn_rsqf(rt2);      // 1 / max(r, R_MIN)
  const float rt = rt2 * ir;
  // dispersion / H-bond and desolvation, inside the 8 A cutoff
  const float ir2 = ir * ir;
  const float ir6 = ir2 * ir2 * ir2;
  const float ir12 = ir6 * ir6;
  const bool hb = HB == 2 && c.y < 0.f;
  const float cy = fabsf(c.y);
  const float irn = hb ? ir6 * ir2 * ir2 : ir6;
  const float nn = hb ? 10.f : 6.f;
  const float a12 = c.x * ir12;
  const float elj = __builtin_fmaf(-cy, irn, a12);
  const float gs = __builtin_amdgcn_exp2f(rt2 * (-1.4426950408889634f / (2.f * kDesolvSigma * kDesolvSigma)));
  const float eds = c.w * gs;
  // electrostatics with the distance-dependent dielectric, inside the 20.48 A cutoff
  const float ex = __builtin_amdgcn_exp2f(rt * (-kDielLambda * kDielB * 1.4426950408889634f));
  const float den = __builtin_fmaf(kDielK, ex, 1.f);
  const float D = __builtin_fmaf(kDielA, den, kDielB);
  const float q = __builtin_amdgcn_rcpf(den * D);
  const float ieps = (den * den) * q;
  const float eel = (c.z * ir) * ieps;
  const bool in1 = r2 < kCutoff * kCutoff, in2 = r2 < kCutoffEl * kCutoffEl;
  const float e = (in1 ? elj + eds : 0.f) + (in2 ? eel : 0.f);
  // (dE/dr) / r of each term: the 12-6 / 12-10 part, the Gaussian's -E / sigma^2, and the
  // electrostatic -E_el (1/r + eps'/eps) / r; zero below R_MIN
  // 12-6: (6 b - 12 a) / r^2 with b = a - elj is -6 (a + elj) / r^2
  const float flj = HB == 0 ? (a12 + elj) * (-6.f * ir2) : __builtin_fmaf(nn * cy, irn, -12.f * a12) * ir2;
  const float flds = __builtin_fmaf(eds, -1.f / (kDesolvSigma * kDesolvSigma), flj);
  const float fel = (__builtin_fmaf(ex * (kDielB * kDielK * kDielLambda * kDielB), q, ir) * -eel) * ir;
  const bool lo = r2 >= kRmin * kRmin;
  f_over_r = (in1 && lo ? flds : 0.f) + (in2 && lo ? fel : 0.f);
  return e;
}

// The pair rows.  Within a lane group no atom occurs twice in a row and a wave's LDS operations
// complete in order, so each lane adds its pair's force, (dE/dr / r)(x_i - x_j) on i and its
// negative on j, into its group's force copy with a plain read-modify-write.  A slot holds the
// byte offsets 4 i | 4 j << 16 of its atoms' entries, so each address is one add.  The H-bond
// pairs sit in the first rows, so the rows after them skip the per-slot choice of the 12-10
// form.  Software pipelined one row deep: a row's force entries and the next row's
// records are requested before the row's arithmetic, the next row's coordinates before its force
// writes (the coordinates are not written here, and the force reads follow the previous row's
// writes in program order); the loop is unrolled by two, and the pair arrays hold one row past
// every span (the next class's first row or a padding row), so the prefetch needs no clamp.
// A two-row-deep pipeline measured slower: its extra registers cost a wave per SIMD.  Each lane
// adds its slots' energies in row order, so the energy-only and gradient paths agree bitwise.
struct P3 {
  float x, y, z;
};

// x, y, z at byte offset `off` of a coordinate or force array of pitch 64A + 1
template <int A>
__device__ __forceinline__ P3 load_p3b(const char* base, uint32_t off) {
  constexpr int P = kWave * A + 1;
  const float* p = reinterpret_cast<const float*>(base + off);
  return P3{p[0], p[P], p[2 * P]};
}

template <int A>
__device__ __forceinline__ void store_p3b(char* base, uint32_t off, P3 v) {
  constexpr int P = kWave * A + 1;
  float* p = reinterpret_cast<float*>(base + off);
  p[0] = v.x;
  p[P] = v.y;
  p[2 * P] = v.z;
}

template <bool GRAD, int HB>
__device__ __forceinline__ float pair_slot(float4 c, P3 xi, P3 xj, P3& fi, P3& fj) {
  const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  float fr;
  const float e = pair_term<HB>(r2, c, fr);
  if (GRAD) {
    const float fx = fr * dx, fy = fr * dy, fz = fr * dz;
    fi.x += fx;
    fi.y += fy;
    fi.z += fz;
    fj.x -= fx;
    fj.y -= fy;
    fj.z -= fz;
  }
  return e;
}

// One row: this row's slot (ij, c) with its coordinates (xi, xj) already loaded; requests the
// next row's slot from (nij, nc) and its coordinates.
template <int A, bool GRAD, int HB>
__device__ __forceinline__ void pair_row(const char* xs, char* fs, uint32_t ij, float4 c, P3 xi, P3 xj,
                                         const uint32_t* nij, const float4* nc, uint32_t& ij_n, float4& c_n,
                                         P3& xi_n, P3& xj_n, float& e) {
  const uint32_t oi = ij & 0xffffu, oj = ij >> 16;
  P3 fi, fj;
  if (GRAD) {
    fi = load_p3b<A>(fs, oi);
    fj = load_p3b<A>(fs, oj);
  }
  ij_n = *nij;
  c_n = *nc;
  e += pair_slot<GRAD, HB>(c, xi, xj, fi, fj);
  xi_n = load_p3b<A>(xs, ij_n & 0xffffu);
  xj_n = load_p3b<A>(xs, ij_n >> 16);
  if (GRAD) {
    store_p3b<A>(fs, oi, fi);
    store_p3b<A>(fs, oj, fj);
  }
}

template <int A, bool GRAD, bool FROM_LDS, int HB>
__device__ __forceinline__ void pair_span(const LigDev& L, const BlockLds& b, int r0, int r1, float& e) {
  if (r0 >= r1) return;
  const int lane = lane_id();
  const uint32_t* pij = (FROM_LDS ? b.pair_ij : L.pair_ij) + lane + (size_t)r0 * kWave;
  const float4* pc = (FROM_LDS ? b.pair_coef : L.pair_coef) + lane + (size_t)r0 * kWave;
  const char* xs = reinterpret_cast<const char*>(b.x);
  // the force copy's byte offset from the coordinates, kept opaque so that no constant part of it
  // is folded into the LDS instructions' offset fields (whose 8-bit dword range the y and z
  // entries would then exceed, costing an address add per atom and row)
  uint32_t fofs = static_cast<uint32_t>(reinterpret_cast<const char*>(b.fg) - xs);
  asm("" : "+v"(fofs));
  char* fs = const_cast<char*>(xs) + fofs;
  uint32_t ij0 = pij[0], ij1;
  float4 c0 = pc[0], c1;
  P3 xi0 = load_p3b<A>(xs, ij0 & 0xffffu), xj0 = load_p3b<A>(xs, ij0 >> 16), xi1, xj1;
  int r = r0;
  for (; r + 2 <= r1; r += 2) {
    pair_row<A, GRAD, HB>(xs, fs, ij0, c0, xi0, xj0, pij + kWave, pc + kWave, ij1, c1, xi1, xj1, e);
    pair_row<A, GRAD, HB>(xs, fs, ij1, c1, xi1, xj1, pij + 2 * kWave, pc + 2 * kWave, ij0, c0, xi0, xj0, e);
    pij += 2 * kWave;
    pc += 2 * kWave;
  }
  if (r < r1) pair_row<A, GRAD, HB>(xs, fs, ij0, c0, xi0, xj0, pij + kWave, pc + kWave, ij1, c1, xi1, xj1, e);
}

// Pair rows [r0, r1): the staged prefix from LDS, the rest from global memory; the rows that may
// hold H-bond pairs [0, mix_rows) first, then the others.  In row order, so every caller adds
// alike.
template <int A, bool GRAD>
__device__ __forceinline__ float pair_rows(const LigDev& L, const BlockLds& b, int r0, int r1) {
  float e = 0.f;
  const int h = L.mix_rows, s = L.pl_rows;
  pair_span<A, GRAD, true, 2>(L, b, r0, min(min(r1, h), s), e);
  pair_span<A, GRAD, false, 2>(L, b, max(r0, s), min(r1, h), e);
  pair_span<A, GRAD, true, 0>(L, b, max(r0, h), min(r1, s), e);
  pair_span<A, GRAD, false, 0>(L, b, max(max(r0, h), s), r1, e);
  return e;
}

// The pair rows [r0, r1) of wave w of the W waves sharing a pose.  Wave a < A also finishes grid
// slot a (atoms 64a + lane), worth about kGridSlotRows rows, so it takes that many fewer rows;
// the last wave takes what remains.  W = 1: all rows.
constexpr int kGridSlotRows = 2;

template <int A, int W>
__device__ __forceinline__ void share_rows(int n_rows, int w, int& r0, int& r1) {
  r0 = 0;
  r1 = n_rows;
  if (W == 1) return;
  const int target = (n_rows + kGridSlotRows * A + W - 1) / W;
  int start = 0;
#pragma unroll
  for (int v = 0; v < W; ++v) {
    const int take = v == W - 1 ? n_rows - start
                                : min(max(target - (v < A ? kGridSlotRows : 0), 0), n_rows - start);
    if (v == w) {
      r0 = start;
      r1 = start + take;
    }
    start += take;
  }
}

// ------------------------------------------------------------------ one pose
// Pieces of a pose evaluation shared by the one-wave and the shared-pose paths.

// Rigid-body genes (wave-uniform): translation, unit quaternion, 1/|q| and the rotation matrix.
struct Rigid {
  float tx, ty, tz, qw, qx, qy, qz, iqn;
  float r00, r01, r02, r10, r11, r12, r20, r21, r22;
};

__device__ __forceinline__ Rigid rigid_of(float xg) {
  Rigid r;
  r.tx = readlane(xg, 0);
  r.ty = readlane(xg, 1);
  r.tz = readlane(xg, 2);
  float qw = readlane(xg, 3), qx = readlane(xg, 4), qy = readlane(xg, 5), qz = readlane(xg, 6);
  r.iqn = __builtin_amdgcn_rsqf(qw * qw + qx * qx + qy * qy + qz * qz);   // 1 / |q|
  qw *= r.iqn;
  qx *= r.iqn;
  qy *= r.iqn;
  qz *= r.iqn;
  r.qw = qw;
  r.qx = qx;
  r.qy = qy;
  r.qz = qz;
  r.r00 = 1.f - 2.f * (qy * qy + qz * qz);
  r.r01 = 2.f * (qx * qy - qw * qz);
  r.r02 = 2.f * (qx * qz + qw * qy);
  r.r10 = 2.f * (qx * qy + qw * qz);
  r.r11 = 1.f - 2.f * (qx * qx + qz * qz);
  r.r12 = 2.f * (qy * qz - qw * qx);
  r.r20 = 2.f * (qx * qz - qw * qy);
  r.r21 = 2.f * (qy * qz + qw * qx);
  r.r22 = 1.f - 2.f * (qx * qx + qy * qy);
  return r;
}

// Torsion gradients: for torsion k (posed axis u_k, posed pivot p_k) the sum over the atoms it
// moves of u_k . ((x - p_k) x F).  With r = x - t and s_k = p_k - t (t the pose's translation,
// so both stay short) that term is u_k . (r x F) - F . (u_k x s_k): each lane forms r x F of its
// atoms once, and per torsion only two dot products remain, with u_k and m_k = u_k x s_k read
// from the wave's torsion table (torsion_axes).  Torsions go in batches of four: each lane forms
// its atoms' terms for the batch's torsions kb..kb+3, then a reduce-scatter with gfx950's
// register-half swaps (no lane addresses, no LDS) leaves the 16 lanes of row r holding parts of
// torsion kb + r's sum -- v_permlane32_swap pairs torsions (kb, kb+2) and (kb+1, kb+3) across the
// wave halves, v_permlane16_swap pairs the results across rows -- and the row's DPP sum (the
// first four steps of wave_sum) completes it.  Gene lane L (torsion tk) reads its torsion's row.
template <int A>
__device__ __forceinline__ float torsion_gradients(const LigDev& L, const AtomRegs<A>& at, int T, const float4* tor,
                                                   const Rigid& rb, const float* x, const float* y, const float* z,
                                                   const float* Fx, const float* Fy, const float* Fz,
                                                   int kb0 = 0, int kb_step = 4) {
  const int tk = at.tor_of_gene;
  float tqx[A], tqy[A], tqz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    const float rx = x[a] - rb.tx, ry = y[a] - rb.ty, rz = z[a] - rb.tz;
    tqx[a] = ry * Fz[a] - rz * Fy[a];
    tqy[a] = rz * Fx[a] - rx * Fz[a];
    tqz[a] = rx * Fy[a] - ry * Fx[a];
  }
  float g = 0.f;
  for (int kb = kb0; kb < T; kb += kb_step) {
    // the batch's four table entries first (the table is padded to a multiple of four torsions),
    // so one wait covers them
    float4 u[4], m[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u[j] = tor[2 * (kb + j)];
      m[j] = tor[2 * (kb + j) + 1];
    }
    // an atom's mask has no bit at or beyond T (k stays below 32: T <= 32, padded to 4)
    float c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kb + j;
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const float ut = u[j].x * tqx[a] + u[j].y * tqy[a] + u[j].z * tqz[a];
        const float t = __builtin_fmaf(-m[j].z, Fz[a], __builtin_fmaf(-m[j].y, Fy[a], __builtin_fmaf(-m[j].x, Fx[a], ut)));
        const float v = __builtin_amdgcn_ubfe(at.mask[a], k, 1) ? t : 0.f;
        c[j] = a == 0 ? v : c[j] + v;
      }
    }
    // lanes 0-31 end with torsion kb (h0) / kb+1 (h1) summed over both halves, lanes 32-63
    // with kb+2 / kb+3
    const auto s0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[0]), __float_as_uint(c[2]), false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[1]), __float_as_uint(c[3]), false, false);
    const float h0 = __uint_as_float(s0[0]) + __uint_as_float(s0[1]);
    const float h1 = __uint_as_float(s1[0]) + __uint_as_float(s1[1]);
    // rows 0, 1, 2, 3 end with torsions kb, kb+1, kb+2, kb+3
    const auto s2 = __builtin_amdgcn_permlane16_swap(__float_as_uint(h0), __float_as_uint(h1), false, false);
    float v = __uint_as_float(s2[0]) + __uint_as_float(s2[1]);
    v += dpp<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141, 0xf>(v);   // row_half_mirror
    v += dpp<0x140, 0xf>(v);   // row_mirror
    const float mine = __shfl(v, ((tk - kb) & 3) * 16, kWave);
    if (tk >= kb && tk < kb + 4) g = mine;
  }
  return g;
}

// Lane k < T writes torsion k's rotation about its reference-frame axis through its reference
// pivot as x -> M x + t (Rodrigues: M = c I + s [u]x + (1 - c) u u^T, t = p - M p) into the wave's
// torsion table, from which the atom loop reads it with broadcast loads.
template <int A>
__device__ __forceinline__ void build_torsion_table(const AtomRegs<A>& at, float4* tor, float xg, int T) {
  const int lane = lane_id();
  const float th = __shfl(xg, at.gene_of_tor, kWave);
  if (lane < T) {
    // v_sin / v_cos take the angle in revolutions
    const float rev = th * 0.15915494309189535f;
    const float sn = __builtin_amdgcn_sinf(rev);
    const float c = __builtin_amdgcn_cosf(rev);
    const float oc = 1.f - c;
    const float ux = at.tux, uy = at.tuy, uz = at.tuz;
    const float m00 = oc * ux * ux + c, m01 = oc * ux * uy - sn * uz, m02 = oc * ux * uz + sn * uy;
    const float m10 = oc * uy * ux + sn * uz, m11 = oc * uy * uy + c, m12 = oc * uy * uz - sn * ux;
    const float m20 = oc * uz * ux - sn * uy, m21 = oc * uz * uy + sn * ux, m22 = oc * uz * uz + c;
    const float vx = at.tpx, vy = at.tpy, vz = at.tpz;
    if constexpr (A == 1) {
      tor[3 * lane + 0] = make_float4(m00, m01, m02, __builtin_fmaf(-m00, vx, __builtin_fmaf(-m01, vy, __builtin_fmaf(-m02, vz, vx))));
      tor[3 * lane + 1] = make_float4(m10, m11, m12, __builtin_fmaf(-m10, vx, __builtin_fmaf(-m11, vy, __builtin_fmaf(-m12, vz, vy))));
      tor[3 * lane + 2] = make_float4(m20, m21, m22, __builtin_fmaf(-m20, vx, __builtin_fmaf(-m21, vy, __builtin_fmaf(-m22, vz, vz))));
    } else {
      tor[3 * lane + 0] = make_float4(m00, m01, m02, vx - (m00 * vx + m01 * vy + m02 * vz));
      tor[3 * lane + 1] = make_float4(m10, m11, m12, vy - (m10 * vx + m11 * vy + m12 * vz));
      tor[3 * lane + 2] = make_float4(m20, m21, m22, vz - (m20 * vx + m21 * vy + m22 * vz));
    }
  }
  wave_sync();
}

// Posed coordinates of this lane's atom slots a with use[a]: torsions from the deepest to the
// root-most (each applied by the lanes whose atom it moves), then orientation and translation.
template <int A>
__device__ __forceinline__ void pose_slots(const LigDev& L, const AtomRegs<A>& at, const float4* tor, const Rigid& rb,
                                           int T, const bool (&use)[A], float (&x)[A], float (&y)[A], float (&z)[A]) {
  float px[A], py[A], pz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    px[a] = at.px[a];
    py[a] = at.py[a];
    pz[a] = at.pz[a];
  }
  // torsion k's transform is applied while torsion k - 1's is being read; for k = 0 that read
  // is of the 48 bytes before the table (the end of this wave's last force copy, inside its LDS),
  // whose values go unused, so the addresses form one stride and need no clamp
  float4 m0 = T > 0 ? tor[3 * (T - 1) + 0] : float4{}, m1 = T > 0 ? tor[3 * (T - 1) + 1] : float4{},
         m2 = T > 0 ? tor[3 * (T - 1) + 2] : float4{};
  for (int k = T - 1; k >= 0; --k) {
    // (two atoms per lane keep the clamped form, which their register allocation prefers)
    const int kn = A == 1 ? k - 1 : max(k - 1, 0);
    const float4 n0 = tor[3 * kn + 0], n1 = tor[3 * kn + 1], n2 = tor[3 * kn + 2];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      if (use[a] && __builtin_amdgcn_ubfe(at.mask[a], k, 1)) {
        // three fused multiply-adds per coordinate, the offset innermost
        const float ox = px[a], oy = py[a], oz = pz[a];
        px[a] = __builtin_fmaf(m0.x, ox, __builtin_fmaf(m0.y, oy, __builtin_fmaf(m0.z, oz, m0.w)));
        py[a] = __builtin_fmaf(m1.x, ox, __builtin_fmaf(m1.y, oy, __builtin_fmaf(m1.z, oz, m1.w)));
        pz[a] = __builtin_fmaf(m2.x, ox, __builtin_fmaf(m2.y, oy, __builtin_fmaf(m2.z, oz, m2.w)));
      }
    }
    m0 = n0;
    m1 = n1;
    m2 = n2;
  }
#pragma unroll
  for (int a = 0; a < A; ++a) {
    x[a] = __builtin_fmaf(rb.r00, px[a], __builtin_fmaf(rb.r01, py[a], __builtin_fmaf(rb.r02, pz[a], rb.tx)));
    y[a] = __builtin_fmaf(rb.r10, px[a], __builtin_fmaf(rb.r11, py[a], __builtin_fmaf(rb.r12, pz[a], rb.ty)));
    z[a] = __builtin_fmaf(rb.r20, px[a], __builtin_fmaf(rb.r21, py[a], __builtin_fmaf(rb.r22, pz[a], rb.tz)));
  }
}

// Sum (and clear) this wave's force copies for this lane's atoms.
template <int A>
__device__ __forceinline__ void sum_force_copies(const LigDev& L, const BlockLds& b, const AtomRegs<A>& at,
                                                 float (&Fx)[A], float (&Fy)[A], float (&Fz)[A]) {
  const int lane = lane_id();
  const int K = L.n_copies;
  const int cs = (int)(lds_coord_bytes(A) / 4);   // floats per copy
#pragma unroll
  for (int a = 0; a < A; ++a) {
    if (at.valid[a]) {
      const int i = lane + kWave * a;
      for (int g = 0; g < K; ++g) {
        float* c = b.f + g * cs;
        const float3 v = load3<A>(c, i);
        Fx[a] += v.x;
        Fy[a] += v.y;
        Fz[a] += v.z;
        store3<A>(c, i, 0.f, 0.f, 0.f);
      }
    }
  }
}

// Gradient components of genes 0..6 (in those lanes, 0 elsewhere).  The translation gradient
// and the torque come from the grid forces alone: intramolecular forces are equal and opposite
// along each pair's line, so they add neither.  Adds the grid forces into F.
template <int A>
__device__ __forceinline__ float rigid_gradient(const Rigid& rb, const float (&x)[A], const float (&y)[A],
                                                const float (&z)[A], const float (&gfx)[A], const float (&gfy)[A],
                                                const float (&gfz)[A], float (&Fx)[A], float (&Fy)[A],
                                                float (&Fz)[A], float e_lane = 0.f, float* E = nullptr) {
  const int lane = lane_id();
  float sfx = 0.f, sfy = 0.f, sfz = 0.f, tqx = 0.f, tqy = 0.f, tqz = 0.f;
#pragma unroll
  for (int a = 0; a < A; ++a) {
    const float rx = x[a] - rb.tx, ry = y[a] - rb.ty, rz = z[a] - rb.tz;
    sfx += gfx[a];
    sfy += gfy[a];
    sfz += gfz[a];
    tqx += ry * gfz[a] - rz * gfy[a];
    tqy += rz * gfx[a] - rx * gfz[a];
    tqz += rx * gfy[a] - ry * gfx[a];
    Fx[a] += gfx[a];
    Fy[a] += gfy[a];
    Fz[a] += gfz[a];
  }
  // the six wave sums as one reduce-scatter (as for the torsion gradients): the half swaps
  // leave rows 0-3 of r0 holding sfx, sfy, sfz, tqx and rows 0 and 2 of r1 holding tqy, tqz,
  // and the row sums complete them
  const auto s0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(sfx), __float_as_uint(sfz), false, false);
  const auto s1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(sfy), __float_as_uint(tqx), false, false);
  const auto s2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(tqy), __float_as_uint(tqz), false, false);
  const float h0 = __uint_as_float(s0[0]) + __uint_as_float(s0[1]);   // sfx | sfz
  const float h1 = __uint_as_float(s1[0]) + __uint_as_float(s1[1]);   // sfy | tqx
  const float h2 = __uint_as_float(s2[0]) + __uint_as_float(s2[1]);   // tqy | tqz
  // with E, the energy rides in the free rows 1 and 3 of r1 (the same tree as wave_sum_rs)
  uint32_t h3 = 0u;
  if (E) {
    const auto s5 = __builtin_amdgcn_permlane32_swap(__float_as_uint(e_lane), __float_as_uint(e_lane), false, false);
    h3 = __float_as_uint(__uint_as_float(s5[0]) + __uint_as_float(s5[1]));
  }
  const auto s3 = __builtin_amdgcn_permlane16_swap(__float_as_uint(h0), __float_as_uint(h1), false, false);
  const auto s4 = __builtin_amdgcn_permlane16_swap(__float_as_uint(h2), h3, false, false);
  float r0 = __uint_as_float(s3[0]) + __uint_as_float(s3[1]);
  float r1 = __uint_as_float(s4[0]) + __uint_as_float(s4[1]);
  r0 += dpp<0xb1, 0xf>(r0);   // quad_perm [1,0,3,2]
  r1 += dpp<0xb1, 0xf>(r1);
  r0 += dpp<0x4e, 0xf>(r0);   // quad_perm [2,3,0,1]
  r1 += dpp<0x4e, 0xf>(r1);
  r0 += dpp<0x141, 0xf>(r0);  // row_half_mirror
  r1 += dpp<0x141, 0xf>(r1);
  r0 += dpp<0x140, 0xf>(r0);  // row_mirror
  r1 += dpp<0x140, 0xf>(r1);
  sfx = readlane(r0, 0);
  sfy = readlane(r0, 16);
  sfz = readlane(r0, 32);
  tqx = readlane(r0, 48);
  tqy = readlane(r1, 0);
  tqz = readlane(r1, 32);
  if (E) *E = readlane(r1, 16);
  const float qw = rb.qw, qx = rb.qx, qy = rb.qy, qz = rb.qz, iqn = rb.iqn;
  float g = 0.f;
  if (lane == 0) g = sfx;
  if (lane == 1) g = sfy;
  if (lane == 2) g = sfz;
  // dE/dq for q/|q| = (w, v): (-2 tau.v, 2 (w tau - v x tau)) / |q|
  if (lane == 3) g = -2.f * (tqx * qx + tqy * qy + tqz * qz) * iqn;
  if (lane == 4) g = 2.f * (qw * tqx - (qy * tqz - qz * tqy)) * iqn;
  if (lane == 5) g = 2.f * (qw * tqy - (qz * tqx - qx * tqz)) * iqn;
  if (lane == 6) g = 2.f * (qw * tqz - (qx * tqy - qy * tqx)) * iqn;
  return g;
}

// Lane k < T: torsion k's posed axis u_k (from the posed coordinates xs of its two atoms) and
// u_k x (p_k - t), p_k its posed pivot and t the pose's translation, into the wave's torsion
// table as tor[2k] and tor[2k + 1] (the posing has finished reading the table's rotations).
template <int A>
__device__ __forceinline__ void torsion_axes(const AtomRegs<A>& at, const float* xs, int T, const Rigid& rb,
                                             float4* tor) {
  const int lane = lane_id();
  if (lane < T) {
    const float3 xa = load3<A>(xs, at.ta), xb = load3<A>(xs, at.tb);
    const float ux = xb.x - xa.x, uy = xb.y - xa.y, uz = xb.z - xa.z;
    const float il = __builtin_amdgcn_rsqf(ux * ux + uy * uy + uz * uz);
    const float nx = ux * il, ny = uy * il, nz = uz * il;
    const float sx = xa.x - rb.tx, sy = xa.y - rb.ty, sz = xa.z - rb.tz;
    tor[2 * lane] = make_float4(nx, ny, nz, 0.f);
    tor[2 * lane + 1] = make_float4(ny * sz - nz * sy, nz * sx - nx * sz, nx * sy - ny * sx, 0.f);
  }
  wave_sync();
}

// Energy (returned, identical in every lane) and, with GRAD, the gradient component of
// gene `lane` (lanes >= n_genes get 0).  xg: gene `lane` of the pose (lanes < n_genes).
// One wave evaluates the pose.
template <int A, int PREC, bool GRAD>
__device__ float eval_pose_one(const LigDev& L, const RecDev& R, const BlockLds& b, const AtomRegs<A>& at,
                               float xg, float& g_out) {
  const int lane = lane_id();
  const int T = L.n_tors;
  const Rigid rb = rigid_of(xg);
  build_torsion_table<A>(at, b.tor, xg, T);
  bool all[A];
#pragma unroll
  for (int a = 0; a < A; ++a) all[a] = true;
  float x[A], y[A], z[A];
  pose_slots<A>(L, at, b.tor, rb, T, all, x, y, z);
#pragma unroll
  for (int a = 0; a < A; ++a) store3<A>(b.x, lane + kWave * a, x[a], y[a], z[a]);

  // grid term: issue the corner loads now, finish after the pair term
  GridFetch gf[A];
  const __amdgpu_buffer_rsrc_t rs = map_rsrc(R);
#pragma unroll
  for (int a = 0; a < A; ++a) grid_fetch<PREC>(R, rs, x[a], y[a], z[a], at.tofs[a], at.q[a], at.valid[a], gf[a]);
  wave_sync();

  // intramolecular pairs; with GRAD each atom then sums (and clears) its force copies
  float e_lane = pair_rows<A, GRAD>(L, b, 0, L.n_rows);
  float Fx[A], Fy[A], Fz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) Fx[a] = Fy[a] = Fz[a] = 0.f;
  if (GRAD) {
    wave_sync();
    sum_force_copies<A>(L, b, at, Fx, Fy, Fz);
  }
  float gfx[A], gfy[A], gfz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) e_lane += grid_finish(R, gf[a], at.valid[a], gfx[a], gfy[a], gfz[a]);
  // one atom per lane: the energy's wave sum rides in the rigid-body reduce-scatter (and the
  // energy-only path sums by the same tree); two atoms per lane: its own sum, which needs fewer
  // live registers at the reduction
  if (!GRAD) return A == 1 ? wave_sum_rs(e_lane) : wave_sum(e_lane);
  float E;
  if constexpr (A != 1) E = wave_sum(e_lane);
  wave_sync();
  float g = A == 1 ? rigid_gradient<A>(rb, x, y, z, gfx, gfy, gfz, Fx, Fy, Fz, e_lane, &E)
                   : rigid_gradient<A>(rb, x, y, z, gfx, gfy, gfz, Fx, Fy, Fz);
  // torsions: every lane forms, for every torsion k, axis . (arm x force) of its atoms that k
  // moves, and reduce-scatters across the wave sum four torsions at a time
  if (T > 0) {
    torsion_axes<A>(at, b.x, T, rb, b.tor);
    const float gk = torsion_gradients<A>(L, at, T, b.tor, rb, x, y, z, Fx, Fy, Fz);
    if (lane >= 7 && lane < L.n_genes) g = gk;
  }
  g_out = g;
  return E;
}

// The same for W > 1 waves (the whole block) sharing one pose; every wave of the block must
// make the same sequence of calls.  Wave a < A poses atom slot a (atoms 64a + lane) into the
// block's coordinate array and issues that slot's grid loads; after a block barrier every wave
// takes its share of the pair rows (share_rows) and wave a finishes grid slot a.  The partial
// forces and energies go to one of two alternating share sets; after a second barrier every
// wave sums them in the same order.  With GRAD, wave w then forms the torsion gradients of the
// torsion batches w, w + W, ... and publishes them by gene; after a third barrier every wave
// holds the same gradient, so the waves take identical search steps.  Hazards: the coordinate
// array and the torsion-gradient array are rewritten only after the barrier that follows their
// last reads; the share sets alternate.
template <int A, int PREC, bool GRAD, int W>
__device__ float eval_pose_shared(const LigDev& L, const RecDev& R, const BlockLds& b, const AtomRegs<A>& at,
                                  float xg, float& g_out, PoseShare& ps) {
  const int lane = lane_id();
  const int T = L.n_tors;
  const int N = L.n_atoms;
  float* X = reinterpret_cast<float*>(b.share);                 // [3][64A + 1] posed coordinates
  unsigned char* sb = reinterpret_cast<unsigned char*>(b.share) + lds_coord_bytes(A);
  float* GG = reinterpret_cast<float*>(sb);                     // [64] torsion gradients by gene lane
  float4* sets = reinterpret_cast<float4*>(sb + 4 * kWave);     // two share sets
  const Rigid rb = rigid_of(xg);

  // pose of this wave's slot (waves >= A have none) and its grid loads
  bool mine[A], gv[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    mine[a] = a == ps.w;
    gv[a] = at.valid[a] && mine[a];
  }
  GridFetch gf[A];
  const __amdgpu_buffer_rsrc_t rs = map_rsrc(R);
  if (ps.w < A) {
    build_torsion_table<A>(at, b.tor, xg, T);
    float x[A], y[A], z[A];
    pose_slots<A>(L, at, b.tor, rb, T, mine, x, y, z);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      if (mine[a]) {
        store3<A>(X, lane + kWave * a, x[a], y[a], z[a]);
        grid_fetch<PREC>(R, rs, x[a], y[a], z[a], at.tofs[a], at.q[a], gv[a], gf[a]);
      } else {
        grid_fetch<PREC>(R, rs, 0.f, 0.f, 0.f, at.tofs[a], at.q[a], false, gf[a]);
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < A; ++a) grid_fetch<PREC>(R, rs, 0.f, 0.f, 0.f, at.tofs[a], at.q[a], false, gf[a]);
  }
  __syncthreads();

  // every atom's posed coordinates (kept for the gradient), this wave's pair rows
  float x[A], y[A], z[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    const float3 v = load3<A>(X, lane + kWave * a);
    x[a] = v.x;
    y[a] = v.y;
    z[a] = v.z;
  }
  BlockLds bs = b;
  bs.x = X;
  int r0, r1;
  share_rows<A, W>(L.n_rows, ps.w, r0, r1);
  float e_lane = pair_rows<A, GRAD>(L, bs, r0, r1);
  float Fx[A], Fy[A], Fz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) Fx[a] = Fy[a] = Fz[a] = 0.f;
  if (GRAD) {
    wave_sync();
    sum_force_copies<A>(L, b, at, Fx, Fy, Fz);
  }
  float gfx[A], gfy[A], gfz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) e_lane += grid_finish(R, gf[a], gv[a], gfx[a], gfy[a], gfz[a]);
  float E = wave_sum(e_lane);

  // publish this wave's partials, meet, take every wave's
  {
    float4* set = sets + (size_t)ps.par * ((size_t)(W + 1) * (N + 1) + W);
    float4* fx = set;                               // [W][N + 1] intramolecular force partials
    float4* gx = set + (size_t)W * (N + 1);         // [N + 1] grid forces
    float4* ew = set + (size_t)(W + 1) * (N + 1);   // [W] energy partials
    if (GRAD) {
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const int i = lane + kWave * a;
        if (at.valid[a]) fx[ps.w * (N + 1) + i] = make_float4(Fx[a], Fy[a], Fz[a], 0.f);
        if (gv[a]) gx[i] = make_float4(gfx[a], gfy[a], gfz[a], 0.f);
      }
    }
    if (lane == 0) ew[ps.w] = make_float4(E, 0.f, 0.f, 0.f);
    __syncthreads();
    E = ew[0].x;
#pragma unroll
    for (int v = 1; v < W; ++v) E += ew[v].x;
    if (GRAD) {
#pragma unroll
      for (int a = 0; a < A; ++a) {
        gfx[a] = gfy[a] = gfz[a] = 0.f;
        if (at.valid[a]) {
          const int i = lane + kWave * a;
          float4 f = fx[i];
#pragma unroll
          for (int v = 1; v < W; ++v) {
            const float4 fv = fx[v * (N + 1) + i];
            f.x += fv.x;
            f.y += fv.y;
            f.z += fv.z;
          }
          Fx[a] = f.x;
          Fy[a] = f.y;
          Fz[a] = f.z;
          const float4 gg = gx[i];
          gfx[a] = gg.x;
          gfy[a] = gg.y;
          gfz[a] = gg.z;
        }
      }
    }
    ps.par ^= 1;
  }
  if (!GRAD) return E;

  float g = rigid_gradient<A>(rb, x, y, z, gfx, gfy, gfz, Fx, Fy, Fz);
  // this wave's torsion batches, published by gene lane, then every wave reads all
  if (T > 0) {
    torsion_axes<A>(at, X, T, rb, b.tor);
    const float gk = torsion_gradients<A>(L, at, T, b.tor, rb, x, y, z, Fx, Fy, Fz, 4 * ps.w, 4 * W);
    const bool gene_t = lane >= 7 && lane < L.n_genes;
    if (gene_t && ((at.tor_of_gene >> 2) % W) == ps.w) GG[lane] = gk;
    __syncthreads();
    if (gene_t) g = GG[lane];
  }
  g_out = g;
  return E;
}

// Dispatch on the waves per pose.
template <int A, int PREC, bool GRAD, int W>
__device__ __forceinline__ float eval_pose(const LigDev& L, const RecDev& R, const BlockLds& b,
                                           const AtomRegs<A>& at, float xg, float& g_out, PoseShare& ps) {
  if constexpr (W == 1) {
    return eval_pose_one<A, PREC, GRAD>(L, R, b, at, xg, g_out);
  } else {
    return eval_pose_shared<A, PREC, GRAD, W>(L, R, b, at, xg, g_out, ps);
  }
}

// ------------------------------------------------------------------ kernels
// One-wave searches keep the register budget of 4 waves per SIMD (one atom per lane) or 3 (two):
// each search is a long dependent chain, and those waves are what hides its latency.
#define MDOCK_SEARCH_OCCUPANCY __attribute__((amdgpu_waves_per_eu(W == 1 ? (A == 1 ? 4 : 3) : 1)))
// Block-size bound of the evaluation kernels: the plan's widest block (16 waves of one atom per
// lane, 12 of two), or 8 waves for the shared-pose instantiations (as before: it caps their
// registers at two waves per SIMD).
#define MDOCK_BLOCK_BOUND_W(A, W) __launch_bounds__((W) == 1 ? kWave * max_waves_per_block(A) : kWave * 8)
#define MDOCK_BLOCK_BOUND(A) __launch_bounds__(kWave * max_waves_per_block(A))

// One block = blockDim / (64 W) poses; W > 1: the block's waves share its one pose.
template <int W>
__device__ __forceinline__ int block_pose(PoseShare& ps) {
  const int wave = threadIdx.x / kWave;
  ps.w = wave % W;
  ps.par = 0;
  return blockIdx.x * (blockDim.x / (kWave * W)) + wave / W;
}

template <int A, int PREC, int W>
__global__ MDOCK_BLOCK_BOUND_W(A, W) void k_eval(LigDev L, RecDev R, int n, const float* __restrict__ genes,
                                                 float* __restrict__ energy, float* __restrict__ grad) {
  const BlockLds b = stage_block<A>(L);
  PoseShare ps;
  const int pose = block_pose<W>(ps);
  if (pose >= n) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const int lane = lane_id();
  const int G = L.n_genes;
  const float xg = lane < G ? genes[(long long)pose * G + lane] : 0.f;
  float g = 0.f;
  float E;
  if (grad) {
    E = eval_pose<A, PREC, true, W>(L, R, b, at, xg, g, ps);
    if (lane < G && ps.w == 0) grad[(long long)pose * G + lane] = g;
  } else {
    E = eval_pose<A, PREC, false, W>(L, R, b, at, xg, g, ps);
  }
  if (lane == 0 && ps.w == 0) energy[pose] = E;
}

// Posed coordinates of this lane's atom slots for the genotype held one gene per lane (xg):
// torsions from the deepest to the root-most about their reference-frame axes (Rodrigues), then
// the unit quaternion's rotation and the translation.  Every lane of the wave must take part.
template <int A>
__device__ __forceinline__ void pose_atoms(const AtomRegs<A>& at, int T, float xg, float (&x)[A], float (&y)[A],
                                           float (&z)[A]) {
  const int lane = lane_id();
  float qw = readlane(xg, 3), qx = readlane(xg, 4), qy = readlane(xg, 5), qz = readlane(xg, 6);
  const float iqn = 1.f / __builtin_sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= iqn; qx *= iqn; qy *= iqn; qz *= iqn;
  const float tx = readlane(xg, 0), ty = readlane(xg, 1), tz = readlane(xg, 2);
  const float th = __shfl(xg, at.gene_of_tor, kWave);
  float tsn = 0.f, tcs = 1.f;
  if (lane < T) sincosf(th, &tsn, &tcs);
  float px[A], py[A], pz[A];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    px[a] = at.px[a];
    py[a] = at.py[a];
    pz[a] = at.pz[a];
  }
  for (int k = T - 1; k >= 0; --k) {
    const float ux = readlane(at.tux, k), uy = readlane(at.tuy, k), uz = readlane(at.tuz, k);
    const float vpx = readlane(at.tpx, k), vpy = readlane(at.tpy, k), vpz = readlane(at.tpz, k);
    const float cs = readlane(tcs, k), sn = readlane(tsn, k);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      if ((at.mask[a] >> k) & 1u) {
        const float vx = px[a] - vpx, vy = py[a] - vpy, vz = pz[a] - vpz;
        const float ud = ux * vx + uy * vy + uz * vz;
        const float cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
        const float omc = (1.f - cs) * ud;
        px[a] = vpx + vx * cs + cx * sn + ux * omc;
        py[a] = vpy + vy * cs + cy * sn + uy * omc;
        pz[a] = vpz + vz * cs + cz * sn + uz * omc;
      }
    }
  }
  const float r00 = 1.f - 2.f * (qy * qy + qz * qz), r01 = 2.f * (qx * qy - qw * qz), r02 = 2.f * (qx * qz + qw * qy);
  const float r10 = 2.f * (qx * qy + qw * qz), r11 = 1.f - 2.f * (qx * qx + qz * qz), r12 = 2.f * (qy * qz - qw * qx);
  const float r20 = 2.f * (qx * qz - qw * qy), r21 = 2.f * (qy * qz + qw * qx), r22 = 1.f - 2.f * (qx * qx + qy * qy);
#pragma unroll
  for (int a = 0; a < A; ++a) {
    x[a] = r00 * px[a] + r01 * py[a] + r02 * pz[a] + tx;
    y[a] = r10 * px[a] + r11 * py[a] + r12 * pz[a] + ty;
    z[a] = r20 * px[a] + r21 * py[a] + r22 * pz[a] + tz;
  }
}

// Writes the posed atoms of one genotype to xyz[n_atoms][3].
template <int A>
__device__ __forceinline__ void store_pose(const LigDev& L, const AtomRegs<A>& at, float xg, float* __restrict__ xyz) {
  float x[A], y[A], z[A];
  pose_atoms<A>(at, L.n_tors, xg, x, y, z);
#pragma unroll
  for (int a = 0; a < A; ++a) {
    if (!at.valid[a]) continue;
    const long long o = (long long)(lane_id() + kWave * a) * 3;
    xyz[o + 0] = x[a];
    xyz[o + 1] = y[a];
    xyz[o + 2] = z[a];
  }
}

// Two atom slots per lane for every ligand size: the same code as the generation epilogue's
// best poses, so both give bitwise the same coordinates for the same genes.
__global__ __launch_bounds__(kBlock) void k_pose(LigDev L, int n, const float* __restrict__ genes,
                                                 float* __restrict__ xyz) {
  const int pose = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (pose >= n) return;
  AtomRegs<2> at;
  load_ligand<2>(L, at);
  const int lane = lane_id();
  const int G = L.n_genes;
  const float xg = lane < G ? genes[(long long)pose * G + lane] : 0.f;
  store_pose<2>(L, at, xg, xyz + (long long)pose * L.n_atoms * 3);
}

// A moved genotype back on its domain: the quaternion (lanes 3..6) renormalised, the torsions
// wrapped to (-pi, pi].
__device__ __forceinline__ float project_gene(float nx, int G) {
  const int lane = lane_id();
  const float q0 = readlane(nx, 3), q1 = readlane(nx, 4), q2 = readlane(nx, 5), q3 = readlane(nx, 6);
  const float iqn = __builtin_amdgcn_rsqf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  if (lane >= 3 && lane < 7) nx = nx * iqn;
  if (lane >= 7 && lane < G) nx = wrap_angle(nx);
  return nx;
}

// ADADELTA step on the gene held by this lane, then the projection.  Returns the new gene.
__device__ __forceinline__ float adadelta_update(float x, float g, float& eg2, float& edx2,
                                                 float rho, float eps, int G) {
  const int lane = lane_id();
  float nx = x;
  if (lane < G) {
    eg2 = rho * eg2 + (1.f - rho) * g * g;
    // the hardware square root and reciprocal square root (about 1 ulp; both arguments are at
    // least eps, far from denormals)
    const float dx = -(__builtin_amdgcn_sqrtf(edx2 + eps) * __builtin_amdgcn_rsqf(eg2 + eps)) * g;
    edx2 = rho * edx2 + (1.f - rho) * dx * dx;
    nx = x + dx;
  }
  return project_gene(nx, G);
}

// ADADELTA from genes_in[row_in] for `iters` steps; the best genotype goes to genes_out[row_out]
// and its energy is returned (wave-uniform).  trace: NULL or [iters] energies of every step;
// trace_x / trace_g: NULL or [iters][G] iterates and gradients of every step.
template <int A, int PREC, int W>
__device__ float local_search_wave(const LigDev& L, const RecDev& R, const BlockLds& b, const AtomRegs<A>& at,
                                   const float* genes_in, long long row_in, float* genes_out,
                                   long long row_out, int iters, float rho, float eps, float* trace,
                                   PoseShare& ps, float* trace_x = nullptr, float* trace_g = nullptr) {
  const int lane = lane_id();
  const int G = L.n_genes;
  float x = lane < G ? genes_in[row_in * G + lane] : 0.f;
  float eg2 = 0.f, edx2 = 0.f;
  float best_x = x;
  float best_e = __builtin_huge_valf();
  for (int it = 0; it < iters; ++it) {
    float g = 0.f;
    const float E = eval_pose<A, PREC, true, W>(L, R, b, at, x, g, ps);
    if (trace && lane == 0 && ps.w == 0) trace[it] = E;
    if (trace_x && lane < G && ps.w == 0) trace_x[(long long)it * G + lane] = x;
    if (trace_g && lane < G && ps.w == 0) trace_g[(long long)it * G + lane] = g;
    if (E < best_e) {
      best_e = E;
      best_x = x;
    }
    x = adadelta_update(x, g, eg2, edx2, rho, eps, G);
  }
  if (lane < G && ps.w == 0) genes_out[row_out * G + lane] = best_x;
  return best_e;
}

// Standalone local search: one pose (W waves) per start genotype.
template <int A, int PREC, int W>
__global__ MDOCK_BLOCK_BOUND_W(A, W) MDOCK_SEARCH_OCCUPANCY void k_local_search(LigDev L, RecDev R, int n,
                                                         const float* genes_in, float* genes_out,
                                                         float* __restrict__ energy_out,
                                                         int iters, float rho, float eps,
                                                         float* __restrict__ trace, float* __restrict__ trace_x,
                                                         float* __restrict__ trace_g) {
  const BlockLds b = stage_block<A>(L);
  PoseShare ps;
  const int job = block_pose<W>(ps);
  if (job >= n) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const long long tg = (long long)job * iters * L.n_genes;
  const float E = local_search_wave<A, PREC, W>(L, R, b, at, genes_in, job, genes_out, job, iters, rho, eps,
                                                trace ? trace + (long long)job * iters : nullptr, ps,
                                                trace_x ? trace_x + tg : nullptr, trace_g ? trace_g + tg : nullptr);
  if (lane_id() == 0 && ps.w == 0) energy_out[job] = E;
}

// ------------------------------------------------------------------ Solis-Wets
// Solis and Wets' adaptive random search (Math. Oper. Res. 6(1), 1981), the local optimiser
// the paper names.  From x with energy E: draw xi ~ N(b, (rho sigma)^2) per gene; move to
// x + xi if its energy is lower, else to x - xi if that is lower.  The bias b becomes
// 0.2 b + 0.4 xi after a + success, b - 0.4 xi after a - success, b / 2 after a double failure;
// rho doubles after 4 successes in a row (at most 4) and halves after 4 failures in a row (at
// least 0.01).  sigma: 0.5 A for translation, 0.05 per quaternion component, 0.25 rad per
// torsion.  Exactly n_evals energy evaluations: the start point, then one or two per step (a
// step the budget cuts short tries x + xi only).  Each step's normals come from Box-Muller on
// two counter-based 24-bit draws per gene, indices 2m and 2m + 1 with m = 64 step + gene.
constexpr float kSwSigmaTrans = 0.5f, kSwSigmaQuat = 0.05f, kSwSigmaTors = 0.25f;
constexpr float kSwRho0 = 1.f, kSwRhoMin = 0.01f, kSwRhoMax = 4.f;
constexpr int kSwExpandAfter = 4, kSwContractAfter = 4;
constexpr int kSwMaxEvals = 1 << 24;   // keeps the draw indices below 2^31

__device__ __forceinline__ float box_muller(uint32_t k1, uint32_t k2) {
  const float u1 = (float)(k1 + 1u) * (1.0f / 16777216.0f);   // (0, 1], exact
  const float u2 = (float)k2 * (1.0f / 16777216.0f);          // [0, 1), exact
  // hardware log2, square root and cosine (the cosine takes revolutions, so cos(2 pi u2) is
  // v_cos(u2)); u1 >= 2^-24 keeps every argument in the normal range
  const float ln_u1 = __builtin_amdgcn_logf(u1) * 0.69314718055994531f;
  return __builtin_amdgcn_sqrtf(-2.f * ln_u1) * __builtin_amdgcn_cosf(u2);
}

// One wave's search from genes_in[row_in]; the final genotype goes to genes_out[row_out] and
// its energy is returned (wave-uniform).  key: draw_prefix of the search's coordinates.
// trace: NULL or [n_evals] energies of every evaluation.
template <int A, int PREC, int W>
__device__ float solis_wets_wave(const LigDev& L, const RecDev& R, const BlockLds& b, const AtomRegs<A>& at,
                                 const float* genes_in, long long row_in, float* genes_out, long long row_out,
                                 int n_evals, uint64_t key, float* trace, PoseShare& ps) {
  const int lane = lane_id();
  const int G = L.n_genes;
  const bool gene = lane < G;
  const float sigma = lane < 3 ? kSwSigmaTrans : (lane < 7 ? kSwSigmaQuat : kSwSigmaTors);
  float x = gene ? genes_in[row_in * G + lane] : 0.f;
  float g;
  const bool out = ps.w == 0;
  float e = eval_pose<A, PREC, false, W>(L, R, b, at, x, g, ps);
  if (trace && lane == 0 && out) trace[0] = e;
  int used = 1;
  float bias = 0.f, rho = kSwRho0;
  int succ = 0, fail = 0;
  for (uint32_t step = 0; used < n_evals; ++step) {
    const uint32_t m = 64u * step + (uint32_t)lane;
    const float z = box_muller(draw_from(key, 2u * m), draw_from(key, 2u * m + 1u));
    const float xi = gene ? bias + rho * sigma * z : 0.f;
    const float x1 = project_gene(x + xi, G);
    const float e1 = eval_pose<A, PREC, false, W>(L, R, b, at, x1, g, ps);
    if (trace && lane == 0 && out) trace[used] = e1;
    ++used;
    bool moved = true;
    if (e1 < e) {
      x = x1;
      e = e1;
      bias = 0.2f * bias + 0.4f * xi;
    } else if (used < n_evals) {
      const float x2 = project_gene(x - xi, G);
      const float e2 = eval_pose<A, PREC, false, W>(L, R, b, at, x2, g, ps);
      if (trace && lane == 0 && out) trace[used] = e2;
      ++used;
      if (e2 < e) {
        x = x2;
        e = e2;
        bias = bias - 0.4f * xi;
      } else {
        bias = 0.5f * bias;
        moved = false;
      }
    } else {
      bias = 0.5f * bias;
      moved = false;
    }
    succ = moved ? succ + 1 : 0;
    fail = moved ? 0 : fail + 1;
    if (succ >= kSwExpandAfter) {
      rho = fminf(kSwRhoMax, 2.f * rho);
      succ = 0;
    }
    if (fail >= kSwContractAfter) {
      rho = fmaxf(kSwRhoMin, 0.5f * rho);
      fail = 0;
    }
  }
  if (gene && out) genes_out[row_out * G + lane] = x;
  return e;
}

// Standalone Solis-Wets: one wave per start genotype; start k draws from coordinates
// (seed, 0, 0, k).
template <int A, int PREC, int W>
__global__ MDOCK_BLOCK_BOUND_W(A, W) MDOCK_SEARCH_OCCUPANCY void k_solis_wets(LigDev L, RecDev R, int n, const float* genes_in,
                                                       float* genes_out, float* __restrict__ energy_out,
                                                       int n_evals, unsigned long long seed,
                                                       float* __restrict__ trace) {
  const BlockLds b = stage_block<A>(L);
  PoseShare ps;
  const int job = block_pose<W>(ps);
  if (job >= n) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const uint64_t key = draw_prefix(seed, 0u, 0u, (uint32_t)job, kPLsSw);
  const float E = solis_wets_wave<A, PREC, W>(L, R, b, at, genes_in, job, genes_out, job, n_evals, key,
                                              trace ? trace + (long long)job * n_evals : nullptr, ps);
  if (lane_id() == 0 && ps.w == 0) energy_out[job] = E;
}

// Initial individual `indiv` of run `run` in the lane-per-gene layout.
__device__ __forceinline__ float initial_gene(const RecDev& R, const GaDev& P, int run, int indiv) {
  const int lane = lane_id();
  const uint64_t sd = P.seed;
  float v = 0.f;
  if (lane < 3) {
    const float lo = lane == 0 ? R.ox : (lane == 1 ? R.oy : R.oz);
    const int nn = lane == 0 ? R.nx : (lane == 1 ? R.ny : R.nz);
    const float hi = lo + (float)(nn - 1) * R.h;
    v = lo + draw_uniform(sd, run, 0, indiv, kPInit, lane) * (hi - lo);
  } else if (lane < 7) {
    const float u1 = draw_uniform(sd, run, 0, indiv, kPInit, 3);
    const float u2 = draw_uniform(sd, run, 0, indiv, kPInit, 4);
    const float u3 = draw_uniform(sd, run, 0, indiv, kPInit, 5);
    const float s1 = __builtin_sqrtf(1.f - u1), s2 = __builtin_sqrtf(u1);
    float sa, ca, sb, cb;
    sincospif(2.f * u2, &sa, &ca);
    sincospif(2.f * u3, &sb, &cb);
    v = lane == 3 ? s1 * sa : (lane == 4 ? s1 * ca : (lane == 5 ? s2 * sb : s2 * cb));
  } else if (lane < P.n_genes) {
    v = kPi - kTwoPi * draw_uniform(sd, run, 0, indiv, kPInit, 6 + (lane - 7));
  }
  return v;
}

// Lowest energy among n, ties to the lower index (wave-uniform result).
__device__ __forceinline__ int wave_argmin(const float* __restrict__ E, int n) {
  const int lane = lane_id();
  float be = __builtin_huge_valf();
  int bi = 0x7fffffff;
  for (int i = lane; i < n; i += kWave) {
    const float e = E[i];
    if (e < be || (e == be && i < bi)) {
      be = e;
      bi = i;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float oe = __shfl_xor(be, off, kWave);
    const int oi = __shfl_xor(bi, off, kWave);
    if (oe < be || (oe == be && oi < bi)) {
      be = oe;
      bi = oi;
    }
  }
  return bi < n ? bi : 0;   // all-NaN input: fall back to index 0, never out of range
}

__device__ __forceinline__ int tournament(const float* __restrict__ E, const GaDev& P, int run,
                                          int gen, int slot, int which) {
  const int a = draw_int(P.pop_size, P.seed, run, gen, slot, kPTournament, 3 * which);
  const int b = draw_int(P.pop_size, P.seed, run, gen, slot, kPTournament, 3 * which + 1);
  const float u = draw_uniform(P.seed, run, gen, slot, kPTournament, 3 * which + 2);
  const float ea = E[a], eb = E[b];
  const int better = (ea < eb || (ea == eb && a <= b)) ? a : b;
  const int worse = better == a ? b : a;
  return u < P.tournament_rate ? better : worse;
}

// Gene unit of gene g: translation components are units 0..2, the quaternion is unit 3,
// torsion k is unit 4 + k.
__device__ __forceinline__ int unit_of(int g) { return g < 3 ? g : (g < 7 ? 3 : g - 3); }

// New individual `slot` of run `run` (slot >= elitism): tournaments, two-point crossover,
// mutation; lane-per-gene layout.
__device__ float offspring_gene(const GaDev& P, const float* __restrict__ genes_in,
                                const float* __restrict__ E, long long rbase, int G, int T, int run,
                                int gen, int slot) {
  const int lane = lane_id();
  const int pa = tournament(E, P, run, gen, slot, 0);
  const int pb = tournament(E, P, run, gen, slot, 1);
  const float xa = lane < G ? genes_in[(rbase + pa) * G + lane] : 0.f;
  const float xb = lane < G ? genes_in[(rbase + pb) * G + lane] : 0.f;
  // two-point crossover over gene units
  float x = xa;
  if (draw_uniform(P.seed, run, gen, slot, kPCrossover, 0) < P.crossover_rate) {
    const int U = 4 + T;
    const int c1 = draw_int(U + 1, P.seed, run, gen, slot, kPCrossover, 1);
    const int c2 = draw_int(U + 1, P.seed, run, gen, slot, kPCrossover, 2);
    const int lo = min(c1, c2), hi = max(c1, c2);
    const int u = unit_of(lane);
    if (u >= lo && u < hi) x = xb;
  }
  // mutation, per unit
  const int m = unit_of(lane < G ? lane : 0);
  const bool mut = lane < G && draw_uniform(P.seed, run, gen, slot, kPMutation, 4 * m) < P.mutation_rate;
  if (mut && m < 3) {
    x += (2.f * draw_uniform(P.seed, run, gen, slot, kPMutation, 4 * m + 1) - 1.f) * P.mut_trans;
  } else if (mut && m >= 4) {
    x = wrap_angle(x + (2.f * draw_uniform(P.seed, run, gen, slot, kPMutation, 4 * m + 1) - 1.f) * P.mut_tors);
  }
  // quaternion unit (identical decision in lanes 3..6): q <- normalise(r (x) q)
  const float cw = readlane(x, 3), cx = readlane(x, 4), cy = readlane(x, 5), cz = readlane(x, 6);
  if (draw_uniform(P.seed, run, gen, slot, kPMutation, 12) < P.mutation_rate) {
    const float alpha = (2.f * draw_uniform(P.seed, run, gen, slot, kPMutation, 13) - 1.f) * P.mut_rot;
    const float zz = 2.f * draw_uniform(P.seed, run, gen, slot, kPMutation, 14) - 1.f;
    const float phi = draw_uniform(P.seed, run, gen, slot, kPMutation, 15);
    const float rxy = __builtin_sqrtf(fmaxf(0.f, 1.f - zz * zz));
    float sp, cp;
    sincospif(2.f * phi, &sp, &cp);
    float sh, ch;
    sincosf(0.5f * alpha, &sh, &ch);
    const float rw = ch, rx = sh * rxy * cp, ry = sh * rxy * sp, rz = sh * zz;
    const float nw = rw * cw - rx * cx - ry * cy - rz * cz;
    const float nx = rw * cx + rx * cw + ry * cz - rz * cy;
    const float ny = rw * cy - rx * cz + ry * cw + rz * cx;
    const float nz = rw * cz + rx * cy - ry * cx + rz * cw;
    const float inv = 1.f / __builtin_sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
    if (lane == 3) x = nw * inv;
    if (lane == 4) x = nx * inv;
    if (lane == 5) x = ny * inv;
    if (lane == 6) x = nz * inv;
  }
  return x;
}

// ------------------------------------------------------------------ GA over a job table
// Every block belongs to one job (blocks[blockIdx.x] = (job, first wave)); a block whose job is
// not in the phase's state leaves before staging anything (uniform per block).

template <int A, int PREC>
__global__ MDOCK_BLOCK_BOUND(A) void k_ga_init(JobDev* __restrict__ jobs, const int2* __restrict__ blocks,
                                                    RecDev R) {
  const int2 bt = blocks[blockIdx.x];
  JobDev& J = jobs[bt.x];
  if (J.state != kJobInit) return;
  const LigDev L = J.L;
  const GaDev P = J.P;
  const BlockLds b = stage_block<A>(L);
  const int w = bt.y + threadIdx.x / kWave;
  if (w >= P.n_runs * P.pop_size) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const int lane = lane_id();
  const int G = L.n_genes;
  const int run = w / P.pop_size, indiv = w % P.pop_size;
  const float x = initial_gene(R, P, run, indiv);
  float g;
  PoseShare ps{0, 0};
  const float E = eval_pose<A, PREC, false, 1>(L, R, b, at, x, g, ps);
  float* genes = J.genes[J.cur];
  if (lane < G) genes[(long long)w * G + lane] = x;
  if (lane == 0) {
    J.energy[J.cur][w] = E;
    J.evals[w] = 1;
  }
}

template <int A, int PREC>
__global__ MDOCK_BLOCK_BOUND(A) void k_ga_generation(JobDev* __restrict__ jobs,
                                                          const int2* __restrict__ blocks, RecDev R) {
  const int2 bt = blocks[blockIdx.x];
  JobDev& J = jobs[bt.x];
  if (J.state != kJobRunning) return;
  const LigDev L = J.L;
  const GaDev P = J.P;
  const int gen = J.gen, cur = J.cur;
  const BlockLds b = stage_block<A>(L);
  const int w = bt.y + threadIdx.x / kWave;
  if (w >= P.n_runs * P.pop_size) return;
  const int lane = lane_id();
  const int G = L.n_genes;
  const int run = w / P.pop_size, slot = w % P.pop_size;
  const long long rbase = (long long)run * P.pop_size;
  const float* genes_in = J.genes[cur];
  float* genes_out = J.genes[cur ^ 1];
  const float* E = J.energy[cur] + rbase;
  float* energy_out = J.energy[cur ^ 1];
  if (slot < P.elitism) {
    const int e = wave_argmin(E, P.pop_size);
    if (lane < G) genes_out[(long long)w * G + lane] = genes_in[(rbase + e) * G + lane];
    if (lane == 0) {
      energy_out[w] = E[e];
      J.evals[w] = 0;
    }
    return;
  }
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const float x = offspring_gene(P, genes_in, E, rbase, G, L.n_tors, run, gen, slot);
  float g;
  PoseShare ps{0, 0};
  const float Enew = eval_pose<A, PREC, false, 1>(L, R, b, at, x, g, ps);
  if (lane < G) genes_out[(long long)w * G + lane] = x;
  if (lane == 0) {
    energy_out[w] = Enew;
    J.evals[w] = 1;
  }
}

// Local-search picks of one run: the n_ls individuals with the lowest random keys (ties to
// the lower index), written as rows in key order.  One wave per run.
__global__ __launch_bounds__(kBlock) void k_ga_ls_pick(JobDev* __restrict__ jobs, const int2* __restrict__ blocks) {
  __shared__ uint32_t keys[kWavesPerBlock][1024];
  const int2 bt = blocks[blockIdx.x];
  JobDev& J = jobs[bt.x];
  if (J.state != kJobRunning) return;
  const GaDev P = J.P;
  const int gen = J.gen;
  const int w = threadIdx.x / kWave;
  const int run = bt.y + w;
  if (run >= P.n_runs || P.n_ls <= 0) return;
  const int lane = lane_id();
  for (int i = lane; i < P.pop_size; i += kWave) keys[w][i] = draw_u24(P.seed, run, gen, i, kPLsPick, 0);
  wave_sync();
  for (int i = lane; i < P.pop_size; i += kWave) {
    const uint32_t ki = keys[w][i];
    int rank = 0;
    for (int j = 0; j < P.pop_size; ++j) {
      const uint32_t kj = keys[w][j];
      rank += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
    }
    if (rank < P.n_ls) J.ls_rows[run * P.n_ls + rank] = run * P.pop_size + i;
  }
}

// Local search on the picked individuals; a block holds blockDim / (64 W) searches from
// (job, first search) of its block-table entry.
template <int A, int PREC, int W>
__global__ MDOCK_BLOCK_BOUND_W(A, W) MDOCK_SEARCH_OCCUPANCY void k_ga_local_search(JobDev* __restrict__ jobs,
                                                            const int2* __restrict__ blocks, RecDev R) {
  const int2 bt = blocks[blockIdx.x];
  JobDev& J = jobs[bt.x];
  if (J.state != kJobRunning) return;
  const LigDev L = J.L;
  const GaDev P = J.P;
  const int cur = J.cur;
  const BlockLds b = stage_block<A>(L);
  PoseShare ps{(int)(threadIdx.x / kWave) % W, 0};
  const int w = bt.y + (int)(threadIdx.x / kWave) / W;
  if (w >= P.n_runs * P.n_ls) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const long long row = J.ls_rows[w];
  float* pop = J.genes[cur ^ 1];
  const float E = local_search_wave<A, PREC, W>(L, R, b, at, pop, row, pop, row, P.ls_iters, P.rho, P.eps,
                                                nullptr, ps);
  if (lane_id() == 0 && ps.w == 0) {
    J.energy[cur ^ 1][row] = E;
    J.evals[row] += P.ls_iters;
  }
}

// Solis-Wets on the picked individuals (Lamarckian write-back); the search of individual i of
// run r in generation g draws from coordinates (seed, r, g, i).
template <int A, int PREC, int W>
__global__ MDOCK_BLOCK_BOUND_W(A, W) MDOCK_SEARCH_OCCUPANCY void k_ga_solis_wets(JobDev* __restrict__ jobs,
                                                          const int2* __restrict__ blocks, RecDev R) {
  const int2 bt = blocks[blockIdx.x];
  JobDev& J = jobs[bt.x];
  if (J.state != kJobRunning) return;
  const LigDev L = J.L;
  const GaDev P = J.P;
  const int cur = J.cur, gen = J.gen;
  const BlockLds b = stage_block<A>(L);
  PoseShare ps{(int)(threadIdx.x / kWave) % W, 0};
  const int w = bt.y + (int)(threadIdx.x / kWave) / W;
  if (w >= P.n_runs * P.n_ls) return;
  AtomRegs<A> at;
  load_ligand<A>(L, at, R.map_stride);
  const int row = J.ls_rows[w];
  const uint64_t key = draw_prefix(P.seed, (uint32_t)(row / P.pop_size), (uint32_t)gen,
                                   (uint32_t)(row % P.pop_size), kPLsSw);
  float* pop = J.genes[cur ^ 1];
  const float E = solis_wets_wave<A, PREC, W>(L, R, b, at, pop, row, pop, row, P.ls_iters, key, nullptr, ps);
  if (lane_id() == 0 && ps.w == 0) {
    J.energy[cur ^ 1][row] = E;
    J.evals[row] += P.ls_iters;
  }
}

// Generation epilogue, one wave per job: the per-run evaluation sum (the miniapp's
// sum_evals), then the job's state advances -- a freshly initialised job starts running, a
// running job swaps its population buffers and moves to the next generation -- and a job whose
// planned generations are done gets its best individual per run.  list: NULL (jobs 0..n-1) or
// [n] entries whose .x is the job.
__global__ __launch_bounds__(kBlock) void k_ga_advance(JobDev* __restrict__ jobs, const int2* __restrict__ list,
                                                       int n_jobs) {
  const int w = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (w >= n_jobs) return;
  JobDev& J = jobs[list ? list[w].x : w];
  const int state = J.state;
  if (state != kJobInit && state != kJobRunning) return;
  const GaDev P = J.P;
  const int lane = lane_id();
  for (int run = 0; run < P.n_runs; ++run) {
    int sum = 0;
    for (int i = lane; i < P.pop_size; i += kWave) sum += J.evals[run * P.pop_size + i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, kWave);
    if (lane == 0) J.evals_of_runs[run] = (state == kJobInit ? 0ll : J.evals_of_runs[run]) + sum;
  }
  int cur = J.cur, gen = J.gen;
  if (state == kJobInit) {
    gen = 1;
  } else {
    cur ^= 1;
    gen += 1;
  }
  const bool done = gen > J.planned;
  if (done) {
    const float* genes = J.genes[cur];
    const float* energy = J.energy[cur];
    const int G = P.n_genes;
    // the best pose's coordinates come from the genes this wave has just picked, in the same
    // pass, so a returned pose always belongs to the returned genotype
    float* bx = J.best_xyz;
    AtomRegs<2> at;
    if (bx) load_ligand<2>(J.L, at);
    for (int run = 0; run < P.n_runs; ++run) {
      const long long base = (long long)run * P.pop_size;
      const int bi = wave_argmin(energy + base, P.pop_size);
      const float xg = lane < G ? genes[(base + bi) * G + lane] : 0.f;
      if (lane < G) J.best_genes[run * G + lane] = xg;
      if (lane == 0) {
        J.best_row[run] = (int)(base + bi);
        J.best_energy[run] = energy[base + bi];
      }
      if (bx) store_pose<2>(J.L, at, xg, bx + (long long)run * J.L.n_atoms * 3);
    }
  }
  if (lane == 0) {
    J.cur = cur;
    J.gen = gen;
    J.state = done ? kJobDone : kJobRunning;
  }
}

// The last node of a captured phase: it follows the join of every size-class branch, so the
// executable graph has this single sink and work queued after the graph's launch on a stream
// is ordered after every branch.
__global__ void k_join() {}

inline unsigned blocks_for(long long waves, int wpb = kWavesPerBlock) {
  return (unsigned)((waves + wpb - 1) / wpb);
}

}  // namespace

// KERNEL<A, PREC> or KERNEL<A, PREC, W> for a ligand of A atoms per lane, maps of precision
// PREC (0 fp32, 1 fp16, 2 bf16) and W waves per pose.
#define MDOCK_LAUNCH_W(KERNEL, A_, P_, W_, GRID, BLK, SM, STREAM, ...)                              \
  switch (W_) {                                                                                   \
    case 2: hipLaunchKernelGGL((KERNEL<A_, P_, 2>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL((KERNEL<A_, P_, 4>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;   \
    default: hipLaunchKernelGGL((KERNEL<A_, P_, 1>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;  \
  }

#define MDOCK_DISPATCH_W(KERNEL, A, PREC, W, GRID, BLK, SM, STREAM, ...)                           \
  do {                                                                                            \
    switch ((PREC) * 2 + ((A) == 2 ? 1 : 0)) {                                                    \
      case 0: MDOCK_LAUNCH_W(KERNEL, 1, 0, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;           \
      case 1: MDOCK_LAUNCH_W(KERNEL, 2, 0, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;           \
      case 2: MDOCK_LAUNCH_W(KERNEL, 1, 1, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;           \
      case 3: MDOCK_LAUNCH_W(KERNEL, 2, 1, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;           \
      case 4: MDOCK_LAUNCH_W(KERNEL, 1, 2, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;           \
      default: MDOCK_LAUNCH_W(KERNEL, 2, 2, W, GRID, BLK, SM, STREAM, __VA_ARGS__) break;          \
    }                                                                                             \
  } while (0)

#define MDOCK_DISPATCH(KERNEL, A, PREC, GRID, BLK, SM, STREAM, ...)                                \
  do {                                                                                            \
    switch ((PREC) * 2 + ((A) == 2 ? 1 : 0)) {                                                    \
      case 0: hipLaunchKernelGGL((KERNEL<1, 0>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;      \
      case 1: hipLaunchKernelGGL((KERNEL<2, 0>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;      \
      case 2: hipLaunchKernelGGL((KERNEL<1, 1>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;      \
      case 3: hipLaunchKernelGGL((KERNEL<2, 1>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;      \
      case 4: hipLaunchKernelGGL((KERNEL<1, 2>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;      \
      default: hipLaunchKernelGGL((KERNEL<2, 2>), GRID, BLK, SM, STREAM, __VA_ARGS__); break;     \
    }                                                                                             \
  } while (0)

#define MDOCK_FN_W(K, A, P) (const void*)K<A, P, 1>, (const void*)K<A, P, 2>, (const void*)K<A, P, 4>
#define MDOCK_FNS_W(K)                                                                            \
  MDOCK_FN_W(K, 1, 0), MDOCK_FN_W(K, 2, 0), MDOCK_FN_W(K, 1, 1), MDOCK_FN_W(K, 2, 1),              \
      MDOCK_FN_W(K, 1, 2), MDOCK_FN_W(K, 2, 2)
#define MDOCK_FNS(K)                                                                              \
  (const void*)K<1, 0>, (const void*)K<2, 0>, (const void*)K<1, 1>, (const void*)K<2, 1>,          \
      (const void*)K<1, 2>, (const void*)K<2, 2>

hipError_t enable_large_lds() {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return hipSuccess;
  const void* fns[] = {MDOCK_FNS_W(k_eval),          MDOCK_FNS_W(k_local_search),  MDOCK_FNS_W(k_solis_wets),
                       MDOCK_FNS_W(k_ga_local_search), MDOCK_FNS_W(k_ga_solis_wets), MDOCK_FNS(k_ga_init),
                       MDOCK_FNS(k_ga_generation)};
  for (const void* f : fns) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsPerBlock);
    if (e != hipSuccess) return e;
  }
  done.insert(dev);
  return hipSuccess;
}

// searches (poses) per block of the ligand's plan
inline int poses_per_block(const LigDev& L) { return std::max(1, L.wpb / std::max(1, L.wpp)); }

hipError_t launch_eval(const LigDev& L, const RecDev& R, int n, const float* genes, float* energy,
                       float* grad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int A = L.n_atoms > kWave ? 2 : 1;
  MDOCK_DISPATCH_W(k_eval, A, R.precision, L.wpp, dim3(blocks_for(n, poses_per_block(L))), dim3(kWave * L.wpb),
                   (size_t)L.lds_bytes, s, L, R, n, genes, energy, grad);
  return hipGetLastError();
}

hipError_t launch_pose(const LigDev& L, int n, const float* genes, float* xyz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pose, dim3(blocks_for(n)), dim3(kBlock), 0, s, L, n, genes, xyz);
  return hipGetLastError();
}

hipError_t launch_local_search(const LigDev& L, const RecDev& R, int n, const float* genes_in,
                               float* genes_out, float* energy_out, int iters, float rho, float eps,
                               float* trace, float* trace_x, float* trace_g, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int A = L.n_atoms > kWave ? 2 : 1;
  MDOCK_DISPATCH_W(k_local_search, A, R.precision, L.wpp, dim3(blocks_for(n, poses_per_block(L))),
                   dim3(kWave * L.wpb), (size_t)L.lds_bytes, s, L, R, n, genes_in, genes_out, energy_out, iters,
                   rho, eps, trace, trace_x, trace_g);
  return hipGetLastError();
}

hipError_t launch_solis_wets(const LigDev& L, const RecDev& R, int n, const float* genes_in, float* genes_out,
                             float* energy_out, int n_evals, unsigned long long seed, float* trace, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_evals < 1 || n_evals > kSwMaxEvals) return hipErrorInvalidValue;
  const int A = L.n_atoms > kWave ? 2 : 1;
  MDOCK_DISPATCH_W(k_solis_wets, A, R.precision, L.wpp, dim3(blocks_for(n, poses_per_block(L))),
                   dim3(kWave * L.wpb), (size_t)L.lds_bytes, s, L, R, n, genes_in, genes_out, energy_out, n_evals,
                   seed, trace);
  return hipGetLastError();
}

hipError_t launch_ga_init(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int lds,
                          const RecDev& R, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  MDOCK_DISPATCH(k_ga_init, A, R.precision, dim3(n_blocks), dim3(kWave * wpb), (size_t)lds, s, jobs, blocks, R);
  return hipGetLastError();
}

hipError_t launch_ga_generation(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int lds,
                                const RecDev& R, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  MDOCK_DISPATCH(k_ga_generation, A, R.precision, dim3(n_blocks), dim3(kWave * wpb), (size_t)lds, s, jobs, blocks,
                 R);
  return hipGetLastError();
}

hipError_t launch_ga_ls_pick(JobDev* jobs, const int2* blocks, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ga_ls_pick, dim3(n_blocks), dim3(kBlock), 0, s, jobs, blocks);
  return hipGetLastError();
}

hipError_t launch_ga_local_search(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int wpp,
                                  int lds, int ls_method, const RecDev& R, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  if (ls_method == kLsSolisWets)
    MDOCK_DISPATCH_W(k_ga_solis_wets, A, R.precision, wpp, dim3(n_blocks), dim3(kWave * wpb), (size_t)lds, s, jobs,
                     blocks, R);
  else
    MDOCK_DISPATCH_W(k_ga_local_search, A, R.precision, wpp, dim3(n_blocks), dim3(kWave * wpb), (size_t)lds, s,
                     jobs, blocks, R);
  return hipGetLastError();
}

hipError_t launch_join(hipStream_t s) {
  hipLaunchKernelGGL(k_join, dim3(1), dim3(kWave), 0, s);
  return hipGetLastError();
}

hipError_t launch_ga_advance(JobDev* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ga_advance, dim3(blocks_for(n_jobs)), dim3(kBlock), 0, s, jobs, (const int2*)nullptr, n_jobs);
  return hipGetLastError();
}

hipError_t launch_ga_advance_list(JobDev* jobs, const int2* list, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ga_advance, dim3(blocks_for(n)), dim3(kBlock), 0, s, jobs, list, n);
  return hipGetLastError();
}

}  // namespace mdock
