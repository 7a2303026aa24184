// Internal structures shared by the host library and the gfx950 kernels of libmdock.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mdock {

constexpr int kWave = 64;
constexpr int kMaxAtoms = 128;
constexpr int kMaxTorsions = 32;
constexpr int kMaxGenes = 7 + kMaxTorsions;
constexpr int kTypes = 7;
constexpr int kMaps = kTypes + 2;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
// Pair records kept in LDS per block; their per-pose force scalars also live in LDS and reach
// the atoms through the incidence table.  Pairs beyond this index (ligands above ~70 atoms)
// are read from global memory and their forces accumulated with LDS atomics.
constexpr int kPairLdsMax = 2048;
constexpr uint32_t kIncNone = 0xffffffffu;

// Scoring constants (AutoDock4 force-field forms and weights).
constexpr float kWvdw = 0.1662f;
constexpr float kWhb = 0.1209f;
constexpr float kWel = 0.1406f;
constexpr float kWds = 0.1322f;
constexpr double kCoulomb = 332.06363;
constexpr float kDielA = -8.5525f;
constexpr float kDielB = 78.4f + 8.5525f;
constexpr float kDielLambda = 0.003627f;
constexpr float kDielK = 7.7839f;
constexpr float kDesolvSigma = 3.6f;
constexpr double kQasp = 0.01097;
constexpr float kRmin = 0.5f;
constexpr float kCutoff = 8.0f;
constexpr float kCutoffEl = 20.48f;
constexpr float kPout = 16384.0f;
constexpr float kKout = 100.0f;

// Ligand constants on the device (views into one allocation).
// Torsions are stored in "internal" order: sorted by the depth of their root-side atom,
// so along any root-to-atom path a larger internal index is a deeper torsion.
struct LigDev {
  int n_atoms, n_tors, n_pairs, n_genes;
  const float4* atom_p0q;     // [N] reference x, y, z (centroid at origin), charge
  const int* atom_type;       // [N]
  const uint32_t* atom_mask;  // [N] bit k set iff torsion k (internal) moves the atom
  const float4* tor_axis;     // [T] unit axis a->b in the reference frame
  const float4* tor_pivot;    // [T] reference position of the root-side atom a
  const int2* tor_ab;         // [T] atoms (a, b)
  const int* tor_gene;        // [T] gene index (7 + caller's torsion index)
  const uint32_t* pair_ij;    // [P] i | j << 8 | hbond << 16
  const float4* pair_coef;    // [P] weighted C12, weighted C6 or C10, W_el*332*qi*qj,
                              //     W_ds*(S_i V_j + S_j V_i)
  int inc_width;              // incidences of the busiest atom (pairs below kPairLdsMax)
  int inc_stride;             // 64 * atoms per lane
  const uint32_t* inc;        // [inc_width][inc_stride]: pair | partner << 16, or kIncNone
};

struct RecDev {
  int nx, ny, nz;
  int precision;              // 0 fp32, 1 fp16, 2 bf16
  float ox, oy, oz;
  float h, inv_h;
  long long map_stride;       // nx*ny*nz
  const void* maps;           // [9][nz][ny][nx]
};

// GA parameters as the kernels see them.
struct GaDev {
  int n_runs, pop_size, n_genes, n_ls, ls_iters, elitism;
  float rho, eps;
  float crossover_rate, mutation_rate, tournament_rate;
  float mut_trans, mut_rot, mut_tors;
  unsigned long long seed;
};

// Host-side ligand after preprocessing (arrays in internal torsion order).
struct LigHost {
  int n_atoms = 0, n_tors = 0, n_genes = 0;
  std::vector<float4> atom_p0q;
  std::vector<int> atom_type;
  std::vector<uint32_t> atom_mask;
  std::vector<float4> tor_axis, tor_pivot;
  std::vector<int2> tor_ab;
  std::vector<int> tor_gene;
  std::vector<uint32_t> pair_ij;
  std::vector<float4> pair_coef;
  int inc_width = 0, inc_stride = 64;
  std::vector<uint32_t> inc;
};

// Returns an empty string on success, else a message; `range_error` tells MD_ERANGE apart.
std::string prepare_ligand(int n_atoms, const float* xyz, const int* type, const float* charge,
                           int n_bonds, const int* bonds, int n_torsions, const int* torsions,
                           int root, int n_types, const float* type_params, LigHost& out,
                           bool& range_error);

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_eval(const LigDev& L, const RecDev& R, int n, const float* genes, float* energy,
                       float* grad, hipStream_t s);
hipError_t launch_pose(const LigDev& L, int n, const float* genes, float* xyz, hipStream_t s);
hipError_t launch_local_search(const LigDev& L, const RecDev& R, int n, const int* rows,
                               const float* genes_in, float* genes_out, float* energy_out,
                               int* evals, int iters, float rho, float eps, float* trace,
                               hipStream_t s);
hipError_t launch_init_population(const LigDev& L, const RecDev& R, const GaDev& P, float* genes,
                                  float* energy, int* evals, hipStream_t s);
hipError_t launch_generation(const LigDev& L, const RecDev& R, const GaDev& P, int gen,
                             const float* genes_in, const float* energy_in, float* genes_out,
                             float* energy_out, int* evals, hipStream_t s);
hipError_t launch_ls_pick(const GaDev& P, int gen, int* rows, hipStream_t s);
hipError_t launch_sum_evals(const GaDev& P, const int* evals, long long* evals_of_runs,
                            hipStream_t s);
hipError_t launch_best_of_runs(const GaDev& P, const float* genes, const float* energy,
                               int* best_row, float* best_energy, float* best_genes,
                               hipStream_t s);

}  // namespace mdock
