/*
 * mdock.h -- C ABI of libmdock, an MI355X (gfx950) implementation of the hot path of
 * AutoDock-style docking as the MiniMDock miniapp captures it: per-pose energy and
 * genotype gradient driving ADADELTA local search inside a Lamarckian genetic
 * algorithm, data-parallel over poses, runs and atoms.
 *
 * Paper passages (arXiv 2203.02096):
 *  - Background, "Design and Structure of MiniMDock": receptor as a 3-D grid
 *    ("reaction field"), ligand as point atoms with self-interactions (H-bonding,
 *    van der Waals, desolvation); degrees of freedom = translation + rotatable bonds
 *    (+ orientation); genetic algorithm with crossover, fitness-based selection and a
 *    Lamarckian local search on a random sample of each generation; several runs of
 *    150 individuals at once, answer = best pose over all runs.
 *  - Section "Approach 1" (listing of decomposed target functions): energy kernel =
 *    per-atom positions, rotations applied in a fixed order, per-atom energy sum.
 *  - Section "Removing architecture-specific code" (sum_evals listings): evaluations
 *    counted per individual and summed per run.
 * The functional forms the paper leaves out follow the AutoDock4 lineage it builds on;
 * each is stated at the entry point that computes it.
 *
 * Conventions
 *  - Every call returns md_status; no exception crosses the ABI.  On error nothing is
 *    written to outputs and no handle is created; md_last_error() gives a message
 *    (thread-local, valid until the next failing call on the same thread).
 *  - Handles are owned by the library and freed by their _destroy call.  _create calls
 *    copy their inputs, so the caller may free them afterwards.
 *  - "dev" pointers are device memory on the current HIP device (e.g. a torch tensor's
 *    data_ptr()), owned by the caller.  "host" pointers are ordinary host memory.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *    that take a stream only enqueue work on it unless stated as blocking.
 *  - Limits: 1 <= n_atoms <= 128, 0 <= n_torsions <= 32 (so n_genes = 7 + n_torsions
 *    <= 39).  Exceeding them returns MD_ERANGE.
 *  - Genotype layout: genes[0:3] translation (Angstrom) of the ligand's reference
 *    centroid; genes[3:7] orientation quaternion (w, x, y, z), used after
 *    normalisation; genes[7:] torsion angles (radians) relative to the input
 *    conformation, right-handed about each rotatable bond taken from its root-side
 *    atom to its far atom, in the order the torsions were given.
 */
#ifndef MDOCK_H
#define MDOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MD_OK = 0,
  MD_EINVAL = -1,     /* malformed argument (null pointer, bad bond graph, bad index, NaN ...) */
  MD_ERANGE = -2,     /* size outside the supported limits */
  MD_ENOMEM = -3,     /* device or host allocation failed */
  MD_EDEVICE = -4,    /* a HIP call failed (no device, launch failure ...) */
  MD_EBUSY = -5,
  MD_ENOTFOUND = -6,
  MD_ECANCELED = -7
} md_status;

typedef enum { MD_MAP_FP32 = 0, MD_MAP_FP16 = 1, MD_MAP_BF16 = 2 } md_map_precision;

typedef struct md_receptor md_receptor;   /* opaque */
typedef struct md_ligand md_ligand;       /* opaque */

/* ------------------------------------------------------------------ receptor grid
 * The receptor's "reaction field" (Background, "Design and Structure of MiniMDock"):
 * n_types atom-type affinity maps, then one electrostatic map (kcal/mol per e) and one
 * desolvation map (kcal/mol per |e|), all sampled on the same grid.  Node (a, b, c) sits
 * at origin + spacing * (a, b, c).
 */
typedef struct {
  int nx, ny, nz;       /* nodes per axis, each >= 2 */
  float spacing;        /* Angstrom, > 0 */
  float origin[3];      /* Angstrom */
  int n_types;          /* number of atom-type maps; must be 7 */
} md_grid_desc;

/* maps: host float32, layout [n_types + 2][nz][ny][nx], finite values.
 * stored: storage precision on the device (FP16/BF16 round to nearest even; the
 * interpolation and everything after it stays FP32).  On the device every grid cell holds its
 * eight corner values per map in one record (the electrostatic and desolvation values side by
 * side, since every atom reads both at the same corners): 72 stored values per node, 288 bytes
 * (FP32) or 144 (FP16/BF16), so that an atom's corners are three aligned runs of memory.
 * The copy is complete when the call returns.  Errors: MD_EINVAL (null/non-finite/bad sizes),
 * MD_ERANGE (FP16 overflow; cell records of 2 GiB or more: above about 7.4M nodes in FP32,
 * 14.9M in FP16/BF16), MD_ENOMEM, MD_EDEVICE. */
md_status md_receptor_create(const md_grid_desc* desc, const float* maps,
                             md_map_precision stored, void* hip_stream, md_receptor** out);
md_status md_receptor_destroy(md_receptor* rec);

/* ------------------------------------------------------------------ ligand
 * Point atoms joined by a connected bond graph (rings allowed inside rigid fragments); the
 * listed bonds are rotatable (degrees of freedom together with translation and orientation;
 * Background, "Design and Structure of MiniMDock") and lie in no ring.  The library moves the reference coordinates so their centroid is the
 * origin, orients each torsion from the root side, finds each torsion's moving set, and
 * builds the intramolecular pair list: pairs at least three bonds apart whose path
 * crosses a rotatable bond.
 *
 * type_params: [n_types][7] float, per type: R_eq (A), eps (kcal/mol), volume (A^3),
 * solvation parameter, H-bond role (0 none, 1 donor, 2 acceptor), R_hb (A), eps_hb.
 */
typedef struct {
  int n_atoms;
  const float* xyz;          /* host [n_atoms][3], Angstrom */
  const int* type;           /* host [n_atoms], in [0, n_types) */
  const float* charge;       /* host [n_atoms], e */
  int n_bonds;               /* n_atoms - 1 (a tree) .. 4 n_atoms */
  const int* bonds;          /* host [n_bonds][2]; connected, no bond twice */
  int n_torsions;
  const int* torsions;       /* host [n_torsions] indices into bonds; each bond must have
                                further atoms on both ends (no terminal bond), lie in no
                                ring, no repeats */
  int root_atom;             /* anchor of the torsion tree, usually 0 */
  int n_types;               /* must be 7 */
  const float* type_params;  /* host [n_types][7] */
} md_ligand_desc;

/* Validates, preprocesses and uploads (synchronously, current device).
 * Errors: MD_EINVAL, MD_ERANGE, MD_ENOMEM, MD_EDEVICE. */
md_status md_ligand_create(const md_ligand_desc* desc, md_ligand** out);
/* MD_EBUSY (nothing freed) while a server request holds the ligand (see md_server_*). */
md_status md_ligand_destroy(md_ligand* lig);
int md_ligand_num_genes(const md_ligand* lig);     /* 7 + n_torsions, or -1 for NULL */
int md_ligand_num_atoms(const md_ligand* lig);
int md_ligand_num_pairs(const md_ligand* lig);     /* intramolecular pairs */

/* Work counts of a prepared ligand, for throughput models: atoms, torsions, intramolecular
 * pairs and the sum over torsions of the number of atoms each one moves.  Any output pointer
 * may be NULL.  Errors: MD_EINVAL (NULL ligand). */
md_status md_ligand_info(const md_ligand* lig, int* n_atoms, int* n_torsions, int* n_pairs,
                         int* sum_moving);

/* ------------------------------------------------------------------ launch plan and autotuner
 * A ligand's launch plan: the evaluation kernels run `waves_per_block` poses per block; each
 * block takes at most `lds_budget` bytes of LDS, which stages the first `staged_rows` of the
 * ligand's `total_rows` rows of 64 intramolecular pair slots (the rest are read from global
 * memory); the lanes of a pair row form conflict-free groups of about n_atoms / group_div lanes
 * (more where the waves' per-group force copies would not fit 160 KiB of LDS).
 * waves_per_pose > 1 (2 or 4) lets that many waves evaluate one pose together in the local
 * searches (md_local_search, md_local_search_sw, md_eval and the docking searches): each takes a
 * share of the pair rows, and their partial forces and energies meet in LDS once per evaluation
 * (one block barrier).  It shortens a search when there are too few searches to fill the device
 * (few runs, large ligands); a block then holds one pose, so waves_per_block becomes
 * waves_per_pose.  The GA's own evaluations keep one wave per pose.
 * A plan changes speed and the order of floating-point sums, not the method: results stay
 * within the parity tolerance of each other and are reproducible for a fixed plan.
 * Defaults: lds_budget 65536, group_div 3, waves_per_block 4, waves_per_pose 1.  Read-only on
 * input to md_ligand_set_plan: lds_bytes, staged_rows, total_rows. */
typedef struct {
  int lds_budget;       /* 0..163840 (gfx950: a block may take the whole 160 KiB LDS of a CU) */
  int group_div;        /* 2..8 */
  int waves_per_block;  /* 1, 2, 4, 8, 12 or 16; ligands of more than 64 atoms take at most 12
                           (larger values are reduced to 12) */
  int lds_bytes, staged_rows, total_rows;   /* outputs: the resulting layout */
  int waves_per_pose;   /* 1 (or 0), 2 or 4 */
} md_plan;
md_status md_ligand_get_plan(const md_ligand* lig, md_plan* out);
/* Re-plans the ligand (host work + one upload; waits for the device to be idle).  The ligand
 * must not be in use by another call.  Errors: MD_EINVAL, MD_ERANGE, MD_EBUSY (a server request
 * holds the ligand), MD_EDEVICE. */
md_status md_ligand_set_plan(md_ligand* lig, const md_plan* plan);

enum { MD_TUNE_FORCE = 1 };   /* time candidates even if the size class is already tuned */
typedef struct {
  md_plan plan;                /* the plan now in the ligand */
  double us_per_eval;          /* its time per local-search evaluation in the tuning launches */
  double default_us_per_eval;  /* the default plan's (0 when taken from the table) */
  int candidates;              /* distinct plans timed */
  int from_table;              /* 1: the class was tuned before; its plan was applied untimed */
} md_tune_info;
/* Autotuner: times the local-search kernel on `rec` for candidate plans -- waves per block
 * {4, 8} x LDS budget {32, 48, 64, 96, 128, 160} KiB, the widest blocks (16 waves, 12 for more
 * than 64 atoms) x {96, 128, 160} KiB, waves per pose {2, 4} x LDS budget {64, 160} KiB, then
 * lane-group sizes N/2 and N/4 for the best -- and applies the fastest to `lig`.  n_starts is the number of local searches one launch
 * will run (md_dock: n_runs x ceil(ls_rate x pop_size)); the candidates are timed on that many
 * random starts inside the box (steps for about 1 ms per launch, best of five launches), since the
 * best plan depends on how well the launch fills the device.  n_starts = 0 (or >= 8192) tunes
 * for launches that fill the device many times over (batches, servers): that plan is also
 * recorded for the ligand's size class (atoms per lane and pair count within a quarter octave),
 * and a later call for a ligand of such a class applies it without timing (unless
 * MD_TUNE_FORCE).  md_ligand_create never consults the record: a new ligand always starts with
 * the default plan, so its results do not depend on what was tuned earlier in the process.  Runs
 * on `hip_stream`, synchronously.  The ligand must not be in use by another call.  info may be
 * NULL.  Errors: MD_EINVAL, MD_ERANGE (n_starts > 2^20), MD_EBUSY (a server request holds the
 * ligand), MD_EDEVICE. */
md_status md_ligand_autotune(const md_receptor* rec, md_ligand* lig, int n_starts, int flags,
                             void* hip_stream, md_tune_info* info);
/* Host only (no device needed): the pair schedule that `plan` gives the ligand `d`, for tests and
 * inspection.  On input plan->lds_budget / group_div / waves_per_block; on output the layout
 * fields.  pair_slots (may be NULL) receives min(capacity, total_rows*64) slots, row-major, each
 * i | j << 8 | hbond << 16 in the library's internal atom order (a pair may appear either way
 * round: the schedule orients each slot to spread the row's LDS accesses over the banks), with
 * bit 17 set for an empty slot (which names atom n_atoms at both ends); *group_lanes (may be
 * NULL) the lanes per conflict-free group.  Errors as md_ligand_create, plus MD_ERANGE for a bad plan. */
md_status md_schedule_preview(const md_ligand_desc* d, md_plan* plan, unsigned* pair_slots, int capacity,
                              int* group_lanes);
md_status md_tune_table_clear(void);   /* forget every tuned size class */
int md_tune_table_size(void);          /* number of tuned size classes */

/* ------------------------------------------------------------------ hot path, one pose
 * Energy and analytic gradient of n_poses genotypes.  Energy = grid part + pair part:
 *  grid part, per atom at grid coordinate g = (x - origin)/spacing: if every
 *    0 <= g_a < n_a - 1, trilinear interpolation of (type map + q*electrostatic +
 *    |q|*desolvation); otherwise 2^14 + 100 d^2 kcal/mol, d = distance to the grid box;
 *  pair part (r clamped below 0.5 A, zero gradient there): 12-6 van der Waals or 12-10
 *    H-bond for donor/acceptor pairs and Gaussian desolvation within 8 A, Coulomb with
 *    the Mehler-Solmajer distance-dependent dielectric within 20.48 A, AutoDock4 weights.
 * Gradient: d/dt = net force, d/dq through the torque and the normalisation (tangent to
 * the unit sphere), d/dtheta_k = axis . sum over moved atoms of arm x force.
 * genes_dev [n_poses][n_genes] f32, energy_dev [n_poses] f32, grad_dev [n_poses][n_genes]
 * f32 or NULL (energy only).  Enqueued on hip_stream.  n_poses may be 0.
 * Errors: MD_EINVAL (null handle/pointer, n_poses < 0), MD_EDEVICE. */
md_status md_eval(const md_receptor* rec, const md_ligand* lig, int n_poses,
                  const float* genes_dev, float* energy_dev, float* grad_dev,
                  void* hip_stream);

/* Posed atom coordinates: xyz_dev [n_poses][n_atoms][3] f32 (receptor frame, Angstrom). */
md_status md_pose(const md_ligand* lig, int n_poses, const float* genes_dev, float* xyz_dev,
                  void* hip_stream);

/* ------------------------------------------------------------------ local search
 * ADADELTA (Zeiler 2012; the gradient-based local search of the AutoDock4 GPU work the
 * paper cites) from each start genotype: per step, evaluate (E, grad) at x, keep x if E
 * is strictly below the best so far, then E[g^2] <- rho E[g^2] + (1-rho) g^2,
 * dx = -sqrt(E[dx^2]+eps)/sqrt(E[g^2]+eps) * g, E[dx^2] <- rho E[dx^2] + (1-rho) dx^2,
 * x += dx, renormalise the quaternion, wrap torsions to (-pi, pi].  n_iters steps cost
 * n_iters evaluations.  Outputs the best genotype and its energy.
 * genes_in_dev/genes_out_dev [n][n_genes] (may alias), energy_out_dev [n];
 * trace_dev: NULL or [n][n_iters] energies of every step.
 * Errors: MD_EINVAL (null, n < 0, n_iters < 1, rho not in [0,1), eps <= 0), MD_EDEVICE. */
md_status md_local_search(const md_receptor* rec, const md_ligand* lig, int n,
                          const float* genes_in_dev, float* genes_out_dev,
                          float* energy_out_dev, int n_iters, float rho, float eps,
                          float* trace_dev, void* hip_stream);

/* md_local_search that also records every step's iterate and gradient, for checking each step
 * of the search on its own (the evaluation at the iterate and the update that leaves it).
 * trace_genes_dev: NULL or [n][n_iters][n_genes], the genotype x_s evaluated at step s;
 * trace_grad_dev: NULL or [n][n_iters][n_genes], the gradient at x_s that the update used.
 * x_{s+1} is trace_genes_dev[s + 1]; the accumulators start at zero as in md_local_search.
 * Same results, arguments and errors as md_local_search otherwise. */
md_status md_local_search_traced(const md_receptor* rec, const md_ligand* lig, int n,
                                 const float* genes_in_dev, float* genes_out_dev,
                                 float* energy_out_dev, int n_iters, float rho, float eps,
                                 float* trace_dev, float* trace_genes_dev, float* trace_grad_dev,
                                 void* hip_stream);

/* Solis-Wets random search (Solis and Wets, Math. Oper. Res. 6(1), 1981; the local optimiser
 * the paper names in Background, "Design and Structure of MiniMDock") from each start
 * genotype.  From x with energy E: xi ~ N(b, (rho sigma)^2) per gene (sigma 0.5 A for the
 * translation, 0.05 per quaternion component, 0.25 rad per torsion); x + xi is taken if its
 * energy is lower, else x - xi if that is lower; b <- 0.2 b + 0.4 xi after a + success,
 * b - 0.4 xi after a - success, b / 2 after a double failure; rho (from 1) doubles after 4
 * successes in a row, at most 4, and halves after 4 failures in a row, at least 0.01.  Moved
 * genotypes get a renormalised quaternion and torsions wrapped to (-pi, pi].  Exactly n_evals
 * energy evaluations: the start point, then one or two per step (a step cut short by the
 * budget tries x + xi only).  Normals: Box-Muller z = sqrt(-2 ln u1) cos(2 pi u2) with
 * u1 = (k1 + 1) / 2^24, u2 = k2 / 2^24 from the counter-based draws (seed, 0, 0, start k,
 * purpose 6, index 2m) and (..., 2m + 1), m = 64 step + gene.  Outputs the final genotype
 * (the lowest energy evaluated) and its energy.
 * genes_in_dev/genes_out_dev [n][n_genes] (may alias), energy_out_dev [n];
 * trace_dev: NULL or [n][n_evals] energies of every evaluation.
 * Errors: MD_EINVAL (null, n < 0, n_evals < 1), MD_ERANGE (n_evals > 2^24), MD_EDEVICE. */
md_status md_local_search_sw(const md_receptor* rec, const md_ligand* lig, int n,
                             const float* genes_in_dev, float* genes_out_dev, float* energy_out_dev,
                             int n_evals, unsigned long long seed, float* trace_dev, void* hip_stream);

/* ------------------------------------------------------------------ docking
 * Lamarckian GA (Background, "Design and Structure of MiniMDock"): n_runs independent runs
 * of pop_size individuals.  Initial individuals: translation uniform in the grid box,
 * uniform random unit quaternion, torsions uniform in (-pi, pi].  Each generation:
 * elitism (best copied to slot 0 when elitism = 1), binary tournaments (better wins with
 * tournament_rate), two-point crossover over the units [t_x, t_y, t_z, q, theta_1..]
 * with crossover_rate, per-unit mutation with mutation_rate (t += U(-mut_trans,
 * mut_trans), q <- normalise(r (x) q) with r a rotation by U(-mut_rot, mut_rot) about a
 * uniform axis, theta += U(-mut_tors, mut_tors)), energy of the new individuals, then
 * a local search of ls_iters evaluations on ceil(ls_rate * pop_size) distinct random
 * individuals, written back: ADADELTA (rho, eps; md_local_search) or Solis-Wets
 * (md_local_search_sw, individual i of run r in generation g drawing from (seed, r, g, i)),
 * chosen by ls_method.  Evaluations are counted per individual and summed per run
 * (sum_evals); a run stops at the first generation boundary where its count reaches
 * max_evals_per_run or max_generations generations have run.  Random numbers:
 * SplitMix64 counter hash of (seed, run, generation, individual, purpose, index).
 */
typedef struct {
  int n_runs, pop_size;
  long long max_evals_per_run;
  int max_generations;
  float ls_rate;
  int ls_iters;
  float rho, eps;
  float crossover_rate, mutation_rate, tournament_rate;
  int elitism;                 /* 0 or 1 */
  float mut_trans, mut_rot, mut_tors;
  unsigned long long seed;
  int ls_method;               /* MD_LS_ADADELTA or MD_LS_SOLIS_WETS (ls_iters <= 2^24) */
} md_dock_params;
enum { MD_LS_ADADELTA = 0, MD_LS_SOLIS_WETS = 1 };

typedef struct {
  int n_runs, n_genes, n_atoms;   /* capacities set by the caller (>= the problem's) */
  float* best_energy;             /* host [n_runs], sorted ascending (ties: lower run) */
  float* best_genes;              /* host [n_runs][n_genes] (row stride = n_genes cap) */
  float* best_xyz;                /* host [n_runs][n_atoms][3] or NULL */
  int* run_index;                 /* host [n_runs] original run of each row, or NULL */
  long long* evals;               /* host [n_runs] or NULL */
  int* generations;               /* host [n_runs] or NULL */
} md_dock_result;

/* Blocking: returns when the results are on the host.  Work runs on hip_stream.
 * Errors: MD_EINVAL (bad parameters or result capacities), MD_ERANGE, MD_ENOMEM,
 * MD_EDEVICE. */
md_status md_dock(const md_receptor* rec, const md_ligand* lig, const md_dock_params* params,
                  md_dock_result* out, void* hip_stream);

/* md_dock without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that forbid it).  Same
 * arguments, results and errors as md_dock, and bitwise the same results (the same kernels),
 * but the dock's workspace lives in a static device array of 8 MiB that every GPU the library
 * runs on holds until the process ends: a dock that needs more (about n_runs * pop_size *
 * (8 * n_genes + 12) bytes plus its results) fails with MD_ERANGE, as does n_runs > 1024.
 * Calls that overlap on one GPU share the array and race: the caller serialises them.  No graph
 * is used, so every generation costs its launches.  Blocking. */
md_status md_dock_noalloc(const md_receptor* rec, const md_ligand* lig, const md_dock_params* params,
                          md_dock_result* out, void* hip_stream);

/* Many docking jobs at once (ligands of different sizes against one receptor): every GA phase
 * is one launch (per atoms-per-lane class) over all jobs, through a device-side job table, so
 * small and large ligands share the GPU.  Each job's result is the same as docking it alone
 * (its random numbers depend only on its own seed and run, generation and individual).
 * Blocking.  Errors: as md_dock, for the first job found invalid (message names it). */
typedef struct {
  const md_ligand* ligand;
  md_dock_params params;
  md_dock_result* result;
} md_dock_job;
md_status md_dock_batch(const md_receptor* rec, int n_jobs, const md_dock_job* jobs, void* hip_stream);

/* Batch autotuner.  In a batch, ligands of different sizes share launches (one per size class
 * and GA phase, as parallel branches of the captured generation), so the plan that is fastest
 * for a ligand alone on the whole device need not be fastest in the mix.  This times whole-batch
 * plan policies on the batch itself -- md_dock_batch of these ligands and parameters, run to
 * generations/3 and to `generations` generations (the shorter of two runs at each length, after
 * a warm-up), the per-generation time being the difference over the extra generations (which
 * leaves out per-call costs) -- and applies the fastest policy
 * to every ligand: MD_POLICY_DEFAULT (every ligand on the default plan),
 * MD_POLICY_TUNED_ALONE (md_ligand_autotune for full-device launches, per size class),
 * MD_POLICY_LDS_ALL (LDS budget 160 KiB: all pair rows staged), MD_POLICY_WIDE_BLOCKS (8 waves
 * per block), MD_POLICY_SMALL_GROUPS (lane groups of about N/2), MD_POLICY_SHARED_LARGE (ligands of
 * more than 64 atoms search with 4 waves per pose, the rest with the default plan: shorter
 * generations for the largest ligands, whose searches set the pace), MD_POLICY_FULL_BLOCKS (the
 * widest blocks -- 16 waves, 12 for more than 64 atoms -- with an LDS budget of 160 KiB: one block
 * per compute unit at full occupancy, all pair rows staged once per block).  The ligands must not be in use
 * by another call.  Blocking.  info may be NULL.  Errors: MD_EINVAL, MD_ERANGE
 * (generations outside [2, 1000]), and md_dock_batch's. */
enum {
  MD_POLICY_DEFAULT = 0, MD_POLICY_TUNED_ALONE = 1, MD_POLICY_LDS_ALL = 2, MD_POLICY_WIDE_BLOCKS = 3,
  MD_POLICY_SMALL_GROUPS = 4, MD_POLICY_SHARED_LARGE = 5, MD_POLICY_FULL_BLOCKS = 6, MD_BATCH_POLICIES = 7
};
typedef struct {
  int policy;                     /* the policy applied */
  int n_policies;
  double ms_per_generation[8];    /* measured per policy (index = policy) */
} md_batch_tune_info;
md_status md_batch_autotune(const md_receptor* rec, int n, md_ligand* const* ligands,
                            const md_dock_params* params, int generations, void* hip_stream,
                            md_batch_tune_info* info);

/* Number of generations md_dock runs for these parameters (all runs share it). */
int md_dock_planned_generations(const md_dock_params* params);

/* ------------------------------------------------------------------ serving
 * Continuous batching for a stream of docking requests against one receptor (the paper's
 * high-throughput screening workflow over many heterogeneous ligands; introduction and its
 * workflow figure).  A worker thread admits queued requests (FIFO) into free slots while their
 * device buffers (populations, counters, results) fit in a pool of hbm_budget_bytes, advances
 * every resident request with the batched GA kernels -- with graphs, each size class of
 * resident ligands by as many generations per tick (up to 8) as fit in the time the most
 * expensive class takes for one; without, one generation per tick -- and retires finished
 * requests at once, freeing their slot and memory for the next admission.  A
 * request's result equals md_dock of the same ligand and parameters.
 * A queued or resident request holds its ligand: until the request has left the device
 * (finished, canceled and out of its slot, or failed), md_ligand_destroy, md_ligand_set_plan
 * and the autotuners refuse that ligand with MD_EBUSY.  Finished requests keep their results
 * and no longer touch the ligand.  The receptor must stay alive until the server is destroyed.
 * Calls are thread-safe.  md_server_destroy drops queued requests, lets resident ones finish,
 * and must not race with md_server_wait on another thread. */
typedef struct md_server md_server;   /* opaque */
typedef struct {
  size_t hbm_budget_bytes;   /* device memory pool for request buffers, >= 1 MiB */
  int max_slots;             /* requests resident at once, 1..4096 */
  int use_graphs;            /* 1 (with md_graphs_enabled()): each tick launches the size
                                classes' chains as parallel branches over several streams;
                                0: one stream, kernel by kernel.  Results are the same. */
} md_server_params;
typedef struct {
  long long ticks, completed;
  int queued, resident;
  size_t pool_used_bytes;
  double busy_seconds;       /* wall time spent running ticks */
} md_server_stats;
/* Errors: MD_EINVAL, MD_ERANGE, MD_ENOMEM, MD_EDEVICE. */
md_status md_server_create(const md_receptor* rec, const md_server_params* params, md_server** out);
/* Queues a request; *ticket identifies it.  MD_ENOMEM if it can never fit the pool. */
md_status md_server_submit(md_server* srv, const md_ligand* lig, const md_dock_params* params,
                           unsigned long long* ticket);
/* *done = 1 once finished (results written to out if non-NULL), canceled or failed
 * (MD_ECANCELED / MD_EDEVICE).  MD_ENOTFOUND for an unknown ticket. */
md_status md_server_poll(md_server* srv, unsigned long long ticket, md_dock_result* out, int* done);
/* Blocks until the request finishes (timeout_s < 0: no limit; MD_EBUSY on timeout). */
md_status md_server_wait(md_server* srv, unsigned long long ticket, md_dock_result* out, double timeout_s);
/* A queued request is canceled at once; a resident one leaves its slot after the current tick
 * and is reported canceled (poll, wait: MD_ECANCELED) only then.  A request that finishes in
 * that tick is reported finished.  Canceling a finished request changes nothing. */
md_status md_server_cancel(md_server* srv, unsigned long long ticket);
/* Host monotonic times (s) of submission, admission to a slot and completion. */
md_status md_server_request_times(md_server* srv, unsigned long long ticket, double* submit_s,
                                  double* start_s, double* end_s);
/* Forgets a finished, canceled or failed request (frees its host-side result); MD_EBUSY while
 * it is queued or on the device (a canceled resident request until it has left its slot). */
md_status md_server_release(md_server* srv, unsigned long long ticket);
md_status md_server_get_stats(md_server* srv, md_server_stats* out);
md_status md_server_destroy(md_server* srv);

/* ------------------------------------------------------------------ kernel timing
 * When enabled, md_dock brackets every kernel it launches with HIP events on its stream and
 * accumulates the elapsed times per kernel kind once the call has synchronised.  Process-wide,
 * not thread-safe; meant for benchmarks.  kind: one of md_kernel_kind. */
typedef enum {
  MD_K_INIT_POPULATION = 0, MD_K_GENERATION = 1, MD_K_LS_PICK = 2, MD_K_LOCAL_SEARCH = 3,
  MD_K_SUM_EVALS = 4, MD_K_BEST_OF_RUNS = 5, MD_K_COUNT = 6
} md_kernel_kind;
md_status md_profile_enable(int on);
md_status md_profile_reset(void);
/* Total milliseconds and number of timed launches of one kernel kind since the last reset. */
md_status md_profile_read(int kind, double* total_ms, long long* launches);

/* HIP graphs for the per-generation launches (default on).  One generation of the LGA is a
 * fixed sequence of launches over the device job table, so md_dock / md_dock_batch capture it
 * once per call and replay it every generation (the server launches the same branches
 * directly, without capture).  Results are identical with graphs off.  Profiling (md_profile_enable)
 * launches kernels one at a time regardless.  Process-wide setting; not thread-safe to change
 * while calls are running. */
md_status md_set_graphs(int on);
int md_graphs_enabled(void);

/* ------------------------------------------------------------------ file front end
 * Readers of the docking program's input files.  The paper docks real small, medium and large
 * ligands against real receptor maps inside a screening workflow (Background, "Design and
 * Structure of MiniMDock"; introduction, workflow figure); these readers turn AutoGrid map files,
 * PDBQT ligands and the atom_par lines of an AutoDock parameter file into the arrays that
 * md_receptor_create and md_ligand_create take.  Host only, no device work.  Errors name the
 * offending line. */

/* One AutoGrid map file held in memory (text, `length` bytes): header records (SPACING s,
 * NELEMENTS nx ny nz -- even interval counts --, CENTER cx cy cz; GRID_PARAMETER_FILE,
 * GRID_DATA_FILE and MACROMOLECULE are accepted and ignored), then one value per line, x
 * fastest, then y, then z.  desc gets nodes per axis (n + 1), the spacing, the minimum corner
 * (CENTER - SPACING * n / 2) and n_types = 7; values [nz][ny][nx] go to `values` (capacity
 * floats; NULL: count only); *n_values (may be NULL) gets the count.  A receptor is nine such
 * maps of one grid, stacked in md_receptor_create's order.  Errors: MD_EINVAL (malformed header
 * or value, value count not (nx+1)(ny+1)(nz+1)), MD_ERANGE (capacity too small). */
md_status md_autogrid_map_parse(const char* text, long long length, md_grid_desc* desc, float* values,
                                long long capacity, long long* n_values);

/* A parsed PDBQT ligand: capacities in, counts and arrays out (caller-owned arrays). */
typedef struct {
  int max_atoms, max_bonds, max_torsions;   /* capacities of the arrays below */
  int n_atoms, n_bonds, n_torsions;         /* set on return (also on MD_ERANGE) */
  int root_atom;                            /* the first atom of the ROOT block: 0 */
  float* xyz;                               /* [max_atoms][3] Angstrom */
  float* charge;                            /* [max_atoms] partial charges, e */
  int* type;                                /* [max_atoms] index into type_names */
  int* bonds;                               /* [max_bonds][2] atom indices */
  int* torsions;                            /* [max_torsions] indices into bonds */
  int* serial;                              /* [max_atoms] the file's serial numbers, or NULL */
} md_pdbqt_ligand;

/* A PDBQT ligand held in memory: ATOM / HETATM records (serial number in columns 7-11,
 * coordinates in columns 31-54, the partial charge and the AutoDock atom type as the record's
 * last two fields), one ROOT block and nested BRANCH a b / ENDBRANCH blocks (a, b serial
 * numbers: a on the root side).  Atoms keep the file's order.  Each atom type is looked up in
 * type_names[n_types] (the receptor's type maps, e.g. {"A","C","HD","N","NA","OA","SA"}).
 * Bonds: atom pairs closer than 1.2 times the sum of their elements' single-bond covalent radii,
 * plus every BRANCH bond; torsions: the BRANCH bonds, in file order.  Rings are allowed inside
 * rigid fragments (md_ligand_create rejects a rotatable bond in a ring).  Errors: MD_EINVAL
 * (malformed or unknown record, atom type without a map or covalent radius, unmatched BRANCH,
 * no ROOT), MD_ERANGE (capacities too small; the counts are set). */
md_status md_pdbqt_parse(const char* text, long long length, int n_types, const char* const* type_names,
                         md_pdbqt_ligand* out);

/* The atom_par records of an AutoDock parameter file held in memory ("atom_par type Rii epsii
 * vol solpar Rij_hb epsij_hb hbond ..."), as md_ligand_desc type_params rows [n_types][7] for
 * the types named in type_names: R_eq = Rii, eps = epsii, volume, solvation parameter, H-bond
 * role (hbond code 0: none, 1-2: donor, 3-5: acceptor), R_hb, eps_hb.  Records of other types
 * are skipped.  Errors: MD_EINVAL (malformed record, a named type without a record). */
md_status md_atom_par_parse(const char* text, long long length, int n_types, const char* const* type_names,
                            float* type_params);

const char* md_last_error(void);
const char* md_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MDOCK_H */
