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
// Pair schedule of a ligand: the intramolecular pairs are laid out in rows of 64 (one pair per
// lane).  The lanes of a row form groups of `group_lanes` consecutive lanes, and within a group
// no atom occurs twice in a row, so every lane can add its pair's force into its group's copy of
// the per-atom force array with a plain read-modify-write (no atomics, no conflicts); the copies
// are summed per atom once per evaluation.  The first `pl_rows` rows are staged in LDS once per
// block; the plan keeps a block's dynamic LDS within kLdsBudget.
constexpr size_t kLdsBudget = 65536;
constexpr uint32_t kPairPad = 1u << 17;   // empty slot of a row: zero coefficients, no force

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
  const uint32_t* pair_ij;    // [n_rows*64] i | j << 8 | hbond << 16 (| kPairPad)
  const float4* pair_coef;    // [n_rows*64] weighted C12, weighted C6 or C10, W_el*332*qi*qj,
                              //     W_ds*(S_i V_j + S_j V_i); zero in empty slots
  int n_rows;                 // rows of 64 pair slots
  int pl_rows;                // rows staged in LDS (a prefix)
  int group_lanes;            // lanes per conflict-free group
  int n_copies;               // force-array copies (groups in use)
  int lds_bytes;              // dynamic LDS of one block
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

// One docking job (ligand + search parameters + its device buffers) in the job table the GA
// kernels read.  gen / cur / state are advanced on the device by the generation epilogue.
enum : int { kJobEmpty = 0, kJobInit = 1, kJobRunning = 2, kJobDone = 3 };

struct JobDev {
  LigDev L;
  GaDev P;
  float* genes[2];            // populations [runs*pop][G]; genes[cur] is the current one
  float* energy[2];           // [runs*pop]
  int* evals;                 // [runs*pop] evaluations of the current generation, per individual
  long long* evals_of_runs;   // [runs] cumulative evaluations
  int* ls_rows;               // [runs*n_ls] rows picked for local search this generation
  int* best_row;              // [runs] outputs once done
  float* best_energy;         // [runs]
  float* best_genes;          // [runs][G]
  int gen;                    // next generation (1-based)
  int cur;                    // index of the current population buffer
  int planned;                // generations to run
  int state;                  // kJob*
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
  std::vector<uint32_t> pair_ij;   // scheduled rows, padded (see LigDev)
  std::vector<float4> pair_coef;
  int n_pairs = 0, n_rows = 0, pl_rows = 0, group_lanes = 64, n_copies = 1, lds_bytes = 0;
};

// LDS layout helpers shared by the host plan and the kernels.
__host__ __device__ inline size_t lds_align16(size_t v) { return (v + 15) & ~size_t(15); }
// per wave: posed coordinates [64*A] and the force-array copies [n_copies][n_atoms], float4 each
__host__ __device__ inline size_t lds_wave_bytes(int n_atoms, int n_copies, int A) {
  return (size_t)16 * kWave * A + (size_t)16 * n_copies * n_atoms;
}
__host__ __device__ inline size_t lds_pairs_bytes(int rows) { return (size_t)rows * kWave * (16 + 4); }

// Returns an empty string on success, else a message; `range_error` tells MD_ERANGE apart.
std::string prepare_ligand(int n_atoms, const float* xyz, const int* type, const float* charge,
                           int n_bonds, const int* bonds, int n_torsions, const int* torsions,
                           int root, int n_types, const float* type_params, LigHost& out,
                           bool& range_error);

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_eval(const LigDev& L, const RecDev& R, int n, const float* genes, float* energy,
                       float* grad, hipStream_t s);
hipError_t launch_pose(const LigDev& L, int n, const float* genes, float* xyz, hipStream_t s);
hipError_t launch_local_search(const LigDev& L, const RecDev& R, int n, const float* genes_in,
                               float* genes_out, float* energy_out, int iters, float rho, float eps,
                               float* trace, hipStream_t s);
// GA phases over a job table.  blocks: [n_blocks] (job, first wave of the block within the
// job's work for this phase).  A: atoms per lane of every job in the table; lds: dynamic LDS.
hipError_t launch_ga_init(JobDev* jobs, const int2* blocks, int n_blocks, int A, int lds,
                          const RecDev& R, hipStream_t s);
hipError_t launch_ga_generation(JobDev* jobs, const int2* blocks, int n_blocks, int A, int lds,
                                const RecDev& R, hipStream_t s);
hipError_t launch_ga_ls_pick(JobDev* jobs, const int2* blocks, int n_blocks, hipStream_t s);
hipError_t launch_ga_local_search(JobDev* jobs, const int2* blocks, int n_blocks, int A, int lds,
                                  const RecDev& R, hipStream_t s);
hipError_t launch_ga_advance(JobDev* jobs, int n_jobs, hipStream_t s);

}  // namespace mdock

// Library handles (opaque to callers of include/mdock.h).
struct md_receptor {
  mdock::RecDev dev{};
  void* d_maps = nullptr;
  int device = 0;
};

struct md_ligand {
  mdock::LigDev dev{};
  void* d_buf = nullptr;
  mdock::LigHost host;
  int device = 0;
};
