// Internal structures shared by the host library and the gfx950 kernels of libmdock.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace mdock {

constexpr int kWave = 64;
constexpr int kMaxAtoms = 128;
constexpr int kMaxTorsions = 32;
constexpr int kMaxGenes = 7 + kMaxTorsions;
constexpr int kTypes = 7;
constexpr int kMaps = kTypes + 2;
// stored values per grid cell record: eight corners of each type map, eight corner pairs of the
// electrostatic and desolvation maps
constexpr int kCellValues = kTypes * 8 + 16;
constexpr int kWavesPerBlock = 4;                  // blocks of the kernels without a ligand plan
constexpr int kBlock = kWave * kWavesPerBlock;
// evaluation kernels: the plan's waves per block; one atom per lane takes at most 128 VGPRs
// (four waves per SIMD, so a block of 16 waves fits a compute unit), two atoms per lane at most
// 168 (three waves per SIMD: blocks of up to 12 waves)
constexpr int kMaxWavesPerBlock = 16;
constexpr int kMaxWavesPerBlock2 = 12;
constexpr int kMaxBlock = kWave * kMaxWavesPerBlock;
__host__ __device__ constexpr int max_waves_per_block(int A) { return A == 1 ? kMaxWavesPerBlock : kMaxWavesPerBlock2; }
// Waves that share one pose in the local-search kernels (1, 2 or 4): the pair rows are split
// between them and their partial forces and energies meet in LDS once per evaluation.  A block
// whose waves share a pose holds exactly that one pose.
constexpr int kMaxWavesPerPose = 4;
constexpr int kMaxLdsPerBlock = 160 * 1024;        // gfx950: all of a compute unit's LDS
// Pair schedule of a ligand: the intramolecular pairs are laid out in rows of 64 (one pair per
// lane).  The lanes of a row form groups of `group_lanes` consecutive lanes, and within a group
// no atom occurs twice in a row, so every lane can add its pair's force into its group's copy of
// the per-atom force array with a plain read-modify-write (no atomics, no conflicts); the copies
// are summed per atom once per evaluation.  An empty slot names atom N (one past the last) at
// both ends with zero coefficients: the coordinate and force arrays have a spare entry there, so
// it needs no branch.  The first `pl_rows` rows are staged in LDS once per block; the plan keeps
// a block's dynamic LDS within kLdsBudget.
constexpr size_t kLdsBudget = 65536;
constexpr uint32_t kPairPad = 1u << 17;   // marks an empty slot (informational)

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
  const int* gene_tor;        // [T] internal torsion of gene 7 + j
  const uint32_t* pair_ij;    // [(n_rows + 1)*64] byte offsets 4 i | 4 j << 16 of the slot's
                              //     atoms in a coordinate or force array; row n_rows is padding
  const float4* pair_coef;    // [(n_rows + 1)*64] weighted C12, weighted C6 or C10, W_el*332*qi*qj,
                              //     W_ds*(S_i V_j + S_j V_i); zero in empty slots
  int n_rows;                 // rows of 64 pair slots
  int mix_rows;               // rows [0, mix_rows) may hold H-bond pairs (the sign of a slot's
                              //     second coefficient marks one), rows [mix_rows, n_rows) hold none
  int pl_rows;                // rows read from LDS (a prefix; one more row is staged behind them)
  int group_lanes;            // lanes per conflict-free group
  int n_copies;               // force-array copies (groups in use)
  int wpb;                    // waves per block of the evaluation kernels
  int wpp;                    // waves per pose of the local-search kernels (1, 2, 4; > 1: wpb == wpp)
  int lds_bytes;              // dynamic LDS of one block
};

struct RecDev {
  int nx, ny, nz;
  int precision;              // 0 fp32, 1 fp16, 2 bf16
  float ox, oy, oz;
  float h, inv_h;
  long long map_stride;       // cell records per type map: nx*ny*nz (a cell is named by its
                              // lowest node, x fastest)
  const void* maps;           // [7][cells][8] type-map corner records, then [cells][8][2]
                              // (electrostatic, desolvation) corner pairs; corner bit 0 +x,
                              // bit 1 +y, bit 2 +z
  unsigned map_bytes;         // bytes of the map allocation (< 2^31: the kernels address it with
                              //     32-bit buffer offsets)
  float gx_max, gy_max, gz_max;   // n - 1 per axis: inside iff 0 <= g < n - 1 (grid units)
  float hx, hy, hz;           // upper corner of the box, origin + (n - 1) h
};

// GA parameters as the kernels see them.
// local optimisers (md_dock_params.ls_method)
enum : int { kLsAdadelta = 0, kLsSolisWets = 1 };

struct GaDev {
  int n_runs, pop_size, n_genes, n_ls, ls_iters, elitism, ls_method;
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
  float* best_xyz;            // [runs][n_atoms][3] posed atoms of best_genes, or NULL
  int gen;                    // next generation (1-based)
  int cur;                    // index of the current population buffer
  int planned;                // generations to run
  int state;                  // kJob*
};

// Tunable choices of a ligand's plan (see plan_ligand).
struct PlanParams {
  int lds_budget = (int)kLdsBudget;   // dynamic LDS of one block, bytes (<= kMaxLdsPerBlock)
  int group_div = 3;                  // lanes per conflict-free group ~ n_atoms / group_div
  int wpb = kWavesPerBlock;           // waves per block (1..max_waves_per_block(A))
  int wpp = 1;                        // waves per pose in the local searches (1, 2, 4; > 1 sets wpb)
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
  std::vector<int> gene_tor;
  std::vector<uint32_t> raw_ij;    // pair list before scheduling
  std::vector<float4> raw_coef;
  std::vector<uint32_t> pair_ij;   // scheduled rows, padded (see LigDev)
  std::vector<float4> pair_coef;
  int n_pairs = 0, n_rows = 0, mix_rows = 0, pl_rows = 0, group_lanes = 64, n_copies = 1, wpb = kWavesPerBlock;
  int wpp = 1;
  int lds_bytes = 0;
  PlanParams plan;
};

// LDS layout helpers shared by the host plan and the kernels.
__host__ __device__ inline size_t lds_align16(size_t v) { return (v + 15) & ~size_t(15); }
// Coordinates and forces are kept as three float arrays (x, y, z) of pitch 64A + 1 (A atoms per
// lane; the last entry is the spare one that empty pair slots name): the pair loop's gathers
// then read 4-byte words at a 4-byte stride, which spreads random atoms over the LDS banks.
__host__ __device__ inline int lds_pitch(int A) { return kWave * A + 1; }
__host__ __device__ inline size_t lds_coord_bytes(int A) { return lds_align16((size_t)12 * lds_pitch(A)); }
// per wave: posed coordinates [3][64A + 1] and the force-array copies [n_copies][3][64A + 1],
// float each (16-byte aligned blocks), then the torsion table [3*roundup4(n_tors)] float4
// (per-pose rotations, later posed axes and pivots; padded so the torsion gradients can read
// whole batches of four)
__host__ __device__ inline size_t lds_wave_bytes(int n_atoms, int n_copies, int A, int n_tors) {
  (void)n_atoms;
  return lds_coord_bytes(A) * (size_t)(1 + n_copies) + (size_t)48 * ((n_tors + 3) & ~3);
}
// rows read from LDS, plus the row behind them that the pair loop's prefetch reads
__host__ __device__ inline int lds_staged_rows(int rows) { return rows > 0 ? rows + 1 : 0; }
__host__ __device__ inline size_t lds_pairs_bytes(int rows) { return (size_t)lds_staged_rows(rows) * kWave * (16 + 4); }
// waves sharing a pose (W > 1): the pose's coordinates [3][64A + 1] (float), its torsion
// gradients by gene lane [64] (float), then two alternating sets (even and odd evaluations) of
// the per-wave intramolecular force partials [W][n_atoms + 1], the grid forces [n_atoms + 1]
// (float4 each) and the per-wave energy partials [W] (one float4 slot each)
__host__ __device__ inline size_t lds_pose_share_bytes(int n_atoms, int W) {
  const int A = n_atoms > kWave ? 2 : 1;
  return W > 1 ? lds_coord_bytes(A) + (size_t)4 * kWave + (size_t)2 * 16 * ((size_t)(W + 1) * (n_atoms + 1) + W)
               : 0;
}

// Returns an empty string on success, else a message; `range_error` tells MD_ERANGE apart.
std::string prepare_ligand(int n_atoms, const float* xyz, const int* type, const float* charge,
                           int n_bonds, const int* bonds, int n_torsions, const int* torsions,
                           int root, int n_types, const float* type_params, LigHost& out,
                           bool& range_error);
// (Re)computes the pair schedule and LDS plan of a prepared ligand.
void plan_ligand(LigHost& h, const PlanParams& pp);

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_eval(const LigDev& L, const RecDev& R, int n, const float* genes, float* energy,
                       float* grad, hipStream_t s);
hipError_t launch_pose(const LigDev& L, int n, const float* genes, float* xyz, hipStream_t s);
// trace: NULL or [n][iters] energies; trace_x, trace_g: NULL or [n][iters][n_genes] iterates
// and gradients of every step
hipError_t launch_local_search(const LigDev& L, const RecDev& R, int n, const float* genes_in,
                               float* genes_out, float* energy_out, int iters, float rho, float eps,
                               float* trace, float* trace_x, float* trace_g, hipStream_t s);
hipError_t launch_solis_wets(const LigDev& L, const RecDev& R, int n, const float* genes_in, float* genes_out,
                             float* energy_out, int n_evals, unsigned long long seed, float* trace, hipStream_t s);
// GA phases over a job table.  blocks: [n_blocks] (job, first wave of the block within the
// job's work for this phase).  A: atoms per lane of every job in the table; lds: dynamic LDS.
hipError_t launch_ga_init(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int lds,
                          const RecDev& R, hipStream_t s);
hipError_t launch_ga_generation(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int lds,
                                const RecDev& R, hipStream_t s);
hipError_t launch_ga_ls_pick(JobDev* jobs, const int2* blocks, int n_blocks, hipStream_t s);
// wpp: waves per search (1, 2, 4); a block holds wpb / wpp searches
hipError_t launch_ga_local_search(JobDev* jobs, const int2* blocks, int n_blocks, int A, int wpb, int wpp,
                                  int lds, int ls_method, const RecDev& R, hipStream_t s);
// Lets every evaluation kernel take up to kMaxLdsPerBlock of dynamic LDS (once per device).
hipError_t enable_large_lds();
hipError_t launch_ga_advance(JobDev* jobs, int n_jobs, hipStream_t s);
// an empty one-wave kernel: the single sink of a captured phase
hipError_t launch_join(hipStream_t s);
// the epilogue for the jobs list[k].x, k < n
hipError_t launch_ga_advance_list(JobDev* jobs, const int2* list, int n, hipStream_t s);

// Per-generation launch schedule over a job table (schedule.cpp).
struct SchedJob {
  int slot;                   // index in the job table
  const LigDev* L;
  int n_runs, pop_size, n_ls, ls_iters, ls_method;
};
// One size class's generation chain: GA generation (+ initial population), local-search picks,
// local search, epilogue -- each a range of the block array (pick blocks cover four runs each,
// epilogue entries name one job each) -- repeated `reps` times per captured phase.
struct ClassChain {
  int A, wpb, wpp, lds, ls_method;
  int pop_first, pop_count, ls_first, ls_count, run_first, run_count, adv_first, adv_count;
  int reps;
  double latency;             // relative serial cost of one generation of the class's slowest job
};
struct GenSchedule {
  std::vector<int2> blocks;   // (slot, first wave) of every block; (slot, 0) epilogue entries
  std::vector<ClassChain> classes;
};
// Optional wrapper around each launch (kind: md_kernel_kind), e.g. for timing.
using LaunchHook = std::function<hipError_t(int, const std::function<hipError_t()>&)>;
// max_reps: 0 -> every class runs `uniform_reps` generations per phase; else each class runs
// about (slowest class's latency / its latency) generations, at most max_reps.
void build_schedule(const std::vector<SchedJob>& jobs, GenSchedule& out, int max_reps = 0, int uniform_reps = 1);
hipError_t launch_init_phase(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                             hipStream_t s, const LaunchHook* hook);
// One generation of every class, kernel by kernel on s (reps ignored).
hipError_t launch_generation_phase(const GenSchedule& g, JobDev* table, const int2* d_blocks,
                                   const RecDev& R, hipStream_t s, const LaunchHook* hook);
// Generations captured as a HIP graph (on private streams) and replayed on any stream.
class GenGraph {
 public:
  GenGraph() = default;
  GenGraph(const GenGraph&) = delete;
  GenGraph& operator=(const GenGraph&) = delete;
  ~GenGraph();
  // each class's chain `reps` times, classes as parallel branches joined at the end
  hipError_t capture(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R);
  // the same work launched directly (no capture) on s and this object's branch streams
  hipError_t launch_direct(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                           hipStream_t s);
  hipError_t launch(hipStream_t s) const;
  // one generation of every class phase by phase (GA generation, local-search picks, local
  // search, epilogue): each phase's class launches run concurrently over s and the branch
  // streams, as in the captured generation, and `hook` brackets the whole phase on s (so a
  // timing hook measures each phase as the classes share the device)
  hipError_t launch_phased(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                           hipStream_t s, const LaunchHook* hook);
  bool ready() const { return exec_ != nullptr; }
  // drops the executable graph (the capture streams stay for the next capture)
  void reset();

 private:
  hipError_t make_streams();
  // fork the classes over `main` and the side streams, each class's chain `reps` times; join
  hipError_t fork_classes(const GenSchedule& g, JobDev* table, const int2* d_blocks, const RecDev& R,
                          hipStream_t main, bool sink);
  hipGraphExec_t exec_ = nullptr;
  // the capture stream, the side streams of the parallel branches and their fork/join events,
  // created on the first capture and kept until the object is destroyed (after the last
  // executable graph captured from them)
  hipStream_t cs_ = nullptr;
  std::vector<hipStream_t> side_;
  std::vector<hipEvent_t> ev_;
};
bool use_graphs();
void set_use_graphs(bool on);

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
  // server requests that may still read the ligand's device buffer (queued or resident); while
  // any does, the ligand is neither destroyed nor re-planned
  mutable std::atomic<int> holds{0};
};

namespace mdock {
// Uploads a prepared ligand (api.cpp): one device allocation, *L gets views into it.
hipError_t upload_ligand(const LigHost& h, void** d_buf, LigDev* L);
}  // namespace mdock
