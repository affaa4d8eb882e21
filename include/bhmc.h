/*
 * bhmc.h - C ABI of the MI355X (gfx950) Barnes-Hut treecode library for
 * single-particle Metropolis Monte Carlo of charged systems (Gan & Xu,
 * "Efficient Implementation of the Barnes-Hut Octree Algorithm for Monte
 * Carlo Simulations of Charged Systems").
 *
 * The calls follow the paper's statement of the method (Sec. 3.3, closing
 * paragraph): locations and charges are given and theta, p and N_0 are
 * prescribed; the octree and the tracking information are built once; every
 * Monte Carlo step evaluates the energy change of the trial move; an accepted
 * move is committed by a local adjustment of the tree; a rejected move leaves
 * the tree unchanged.
 *
 * Conventions shared by every call
 *   - Floating point is IEEE FP64 throughout; the energy change that feeds the
 *     Metropolis test is accumulated in FP64.
 *   - Energies are in units of k_B T: l_B absorbs beta and the solvent
 *     permittivity (eq. 2.1).  Charges are valences.
 *   - "dev" pointers are device pointers on the current HIP device, "host"
 *     pointers are host memory.  Arrays are contiguous, one value per ion,
 *     in ion order 0..N-1.  Input arrays stay owned by the caller and are
 *     copied at build time; output arrays are owned by the caller.
 *   - A tree handle and all its device memory belong to the library until
 *     bhmc_free.  Every call enqueues its work on the stream given at build;
 *     a call that returns a host value synchronises that stream first.
 *   - A non-OK status leaves the tree as it was, and bhmc_last_error()
 *     returns a message for the calling thread.
 *   - Ion indices are 0..N-1.  Kelvin images are internal sources N..2N-1 and
 *     are never addressed by the caller.
 */
#ifndef BHMC_H
#define BHMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BHMC_OK = 0,
    BHMC_EINVAL = -1,     /* bad argument or parameter                       */
    BHMC_EOUTSIDE = -2,   /* an ion outside the confinement, or a source outside the root cube */
    BHMC_EOVERLAP = -3,   /* a committed move that overlaps a hard core       */
    BHMC_ENOMEM = -4,     /* device allocation failed                         */
    BHMC_EHIP = -5,       /* a HIP runtime call failed                        */
    BHMC_ECAPACITY = -6,  /* a leaf's index array is full (see bhmc_commit_move) */
    BHMC_ESTACK = -7,     /* a traversal list outgrew its capacity (see bhmc_set_frontier_capacity) */
    BHMC_EINTERNAL = -8   /* a device-side index check failed; the handle must be freed */
} bhmc_status;

/* Rejection reasons reported with an infinite energy change. */
enum { BHMC_REASON_NONE = 0, BHMC_REASON_WALL = 1, BHMC_REASON_OVERLAP = 2 };

/* Physical and numerical parameters of one system.
 *   l_B        Bjerrum length (eq. 2.1).
 *   theta      MAC parameter, 0 <= theta < 1: a cell is used through its
 *              multipole expansion iff rho_A / r_{i,A} <= theta and
 *              N_A >= n0 (Sec. 3.2); rho_A is half the cell diagonal.
 *   p          expansion order of eq. 3.3, 0 <= p <= 10.
 *   leaf_cap   a cell is split into its eight children iff it holds more than
 *              leaf_cap sources and its level is below max_depth (adaptive
 *              form of the bisection of Sec. 3.2; leaf_cap = 0 with
 *              max_depth = L_max is the paper's uniform tree over occupied
 *              cells).
 *   n0         minimum expansion number N_0 (Sec. 3.2); 0 disables it.
 *   max_depth  deepest level, 0..21 (21 bits per axis in the keys).
 *   geom       0: confinement and root are the cube [box_lo, box_lo + side)^3.
 *              1: spherical cell (Sec. 4): ions confined to r_min < |r| < r_max
 *                 around a fixed central charge Q_center; the root cube
 *                 [box_lo, box_lo + side)^3 must contain the shell.
 *   images     1: one Kelvin image per ion inside the dielectric sphere of
 *              radius a (requires geom = 1): charge gamma a q / |r| at
 *              a^2 r / |r|^2, gamma = (eps_out - eps_in) / (eps_out + eps_in).
 *   hard_core  contact distance tau: a move to within tau of another ion
 *              (distance <= tau) is rejected (eq. 2.1).  0 = point charges
 *              (a move onto another ion is then rejected as an overlap).
 *   slot_slack capacity of a leaf's index array is
 *              slot_slack * max(count at build, leaf_cap) + 2 + line_images
 *              (one move inserts at most the ion and its images).
 *   far_fp32   1: the expansions of eq. 3.3 in the traversals of the energy,
 *              the energy change and the Metropolis kernels use a single-
 *              precision copy of the moments and single-precision Taylor
 *              coefficients (eq. 3.4) per far cell, each cell's value then
 *              added to the potential in FP64 (the energy change that feeds
 *              the Metropolis test is accumulated in FP64; near sources, the
 *              moments themselves and their repair stay FP64).  The rounding
 *              this adds is at most about (C(p+3,3) + 3p + 4) 2^-24 times the
 *              far field's magnitude sum_A sum_n |T_n M_A^n|.  The gradient is
 *              always FP64.  0: everything in FP64.
 *   line_images 0, or M in 1..8 (needs images = 1, n0 = 0, eps_in <= eps_out):
 *              the multiple-image model of the dielectric sphere that the paper
 *              names in Sec. 1 and Sec. 5.  The exact reaction potential of a
 *              charge outside the sphere is that of the Kelvin image plus a line
 *              of charge from the centre to the Kelvin point r_K, of density
 *              -sigma q_K t^(sigma-1) at t r_K (t in [0, 1], sigma =
 *              eps_out / (eps_in + eps_out)); the line is replaced by the M-point
 *              Gauss rule of the weight t^(sigma-1) on [0, 1] (nodes t_m and
 *              weights w_m rounded to multiples of 2^-40): M more sources per
 *              ion, -sigma w_m q_K at t_m r_K, numbered 2n + m n + i.  Every
 *              call evaluates it: a move moves the ion, its Kelvin image and
 *              its M line images, in that order (the Metropolis calls then
 *              take one move per traversal), and the gradient maps each line
 *              image back to its ion through t_m r_K and -sigma w_m q_K.
 *   reserved   0.
 */
typedef struct {
    double l_B;
    double theta;
    int32_t p;
    int32_t leaf_cap;
    int32_t n0;
    int32_t max_depth;
    int32_t geom;
    int32_t images;
    double box_lo[3];
    double box_side;
    double a;
    double Q_center;
    double eps_in, eps_out;
    double r_min, r_max;
    double hard_core;
    int32_t slot_slack;
    int32_t far_fp32;
    int32_t line_images;
    int32_t reserved;   /* 0 */
} bhmc_params;

/* Statistics of a Monte Carlo run, summed over the moves it made. */
typedef struct {
    int64_t moves;          /* trial moves evaluated                          */
    int64_t accepted;
    int64_t rejected_wall;  /* left the confinement (Sec. 4)                  */
    int64_t rejected_overlap; /* hard-core overlap (eq. 2.1)                  */
    int64_t rejected_metropolis;
    int64_t rebuilds;       /* rebuilds forced by a full leaf index array     */
} bhmc_stats;

typedef struct bhmc_tree bhmc_tree;

/* Tree geometry summary for one replica. */
typedef struct {
    int64_t n;        /* ions                                                 */
    int64_t nsrc;     /* sources: n, or (2 + line_images) n with images       */
    int64_t ncell;
    int64_t nleaf;
    int64_t nterms;   /* (p+1)(p+2)(p+3)/6 moments per cell                   */
    int64_t depth;    /* deepest level present                                */
    int64_t pool;     /* leaf index-array slots allocated                     */
} bhmc_info;

/* Build the octree, tracking information and moments of one system
 * (Sec. 3.2, Sec. 3.3).  x, y, z, q: dev, n values each.  hip_stream: a
 * hipStream_t (NULL = default stream).  Errors: EINVAL for bad parameters,
 * EOUTSIDE if an ion violates the confinement or a source lies outside the
 * root cube, ENOMEM, EHIP. */
bhmc_status bhmc_build(const bhmc_params* params, int64_t n, const double* x, const double* y,
                       const double* z, const double* q, void* hip_stream, bhmc_tree** out);

/* Build R independent replicas in one handle (one tree each).  params: host
 * array of R parameter sets; all must share p.  n_per_replica: host, R
 * values.  x, y, z, q: dev, the replicas' ions concatenated in replica order.
 * Replica r is addressed by its index in the calls below. */
bhmc_status bhmc_batch_create(const bhmc_params* params, int32_t R, const int64_t* n_per_replica,
                              const double* x, const double* y, const double* z, const double* q,
                              void* hip_stream, bhmc_tree** out);

void bhmc_free(bhmc_tree* tree);

/* Number of replicas in the handle (1 for bhmc_build). */
int32_t bhmc_replicas(const bhmc_tree* tree);

bhmc_status bhmc_info_get(bhmc_tree* tree, int32_t replica, bhmc_info* info);

/* Treecode total energy of replica `replica` (host result):
 *   E = l_B [ 1/2 sum_i q_i phi_i(r_i) + 1/2 sum_i gamma a q_i^2 / (|r_i|^2 - a^2)
 *             + Q_center sum_i q_i / |r_i| ],
 * phi_i = potential at r_i from every source except ion i and its image,
 * evaluated by the MAC traversal of Sec. 3.2 with the expansion of eq. 3.3.
 * phi_dev (nullable): dev, n values, receives phi_i. */
bhmc_status bhmc_energy(bhmc_tree* tree, int32_t replica, double* E_host, double* phi_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy of
 * bhmc_energy without any allocation or host synchronisation.  The per-ion
 * energy terms are kept in a fixed device array of the library (4 MiB per
 * device, held until the process ends), so replicas of at most 524,288 ions
 * are accepted (EINVAL beyond).  E_dev: dev, 1 value, receives E; phi_dev
 * (nullable): dev, n values.  Work is enqueued on the handle's stream and the
 * call returns at once; a traversal that failed leaves NaN in *E_dev (host
 * errors are returned as usual).  Every handle on a device shares the one
 * array, which keeps the last call's contents: calls that overlap on one
 * device (concurrent streams or threads) race. */
bhmc_status bhmc_energy_noalloc(bhmc_tree* tree, int32_t replica, double* E_dev, double* phi_dev);

/* Energy change of moving ion i of replica 0 to r_new (host, 3 values), on
 * the committed tree (Sec. 1: the particle's energy evaluated twice):
 *   dE = l_B q_i [phi(r_new) - phi(r_i)] + exact self-image change
 *        + exact central-charge change,
 * phi from every source except ion i and its images (the self-image change
 * includes ion i's own line images).  A move out of the confinement or onto
 * a hard core gives dE = +inf and *reason_host = BHMC_REASON_WALL /
 * BHMC_REASON_OVERLAP (not an error).  The tree is not modified. */
bhmc_status bhmc_delta_energy(bhmc_tree* tree, int64_t i, const double* r_new, double* dE_host,
                              int32_t* reason_host);

/* Commit the move of ion i of replica 0 to r_new (host, 3 values) by the
 * local adjustment of Sec. 3.3: ion then image (then the line images, in
 * source order) are moved between leaf index
 * arrays (delete = last entry fills the hole; add = append) and their old and
 * new contributions are removed from / added to the moments and counts of
 * every ancestor cell.  EINVAL if the move leaves the confinement,
 * EOVERLAP if it overlaps a hard core, ECAPACITY if a leaf index array is
 * full (call bhmc_rebuild, then commit again).  The tree is unchanged on
 * error. */
bhmc_status bhmc_commit_move(bhmc_tree* tree, int64_t i, const double* r_new);

/* Run n_moves Metropolis moves move0 .. move0+n_moves-1 of replica `replica`
 * entirely on the device (Sec. 2 steps 1-3; Sec. 3.3).  Move m draws twelve
 * Philox4x32-10 words (Salmon et al., SC'11) with key (lo32 seed, hi32 seed)
 * and counters (lo32 m, hi32 m, replica, t), t = 0, 1, 2:
 *   ion  i = (w0 * N) >> 32,
 *   displacement_d = step * (u_d - 1/2) with u_x, u_y, u_z from (w2,w3),
 *   (w4,w5), (w6,w7) and u(a,b) = ((a >> 5) 2^26 + (b >> 6)) 2^-53,
 *   alpha = u(w8, w9);
 * accept iff dE <= 0 or alpha <= exp(-dE).  If an accepted move would
 * overflow a leaf index array, the replica's tree is rebuilt from its current
 * positions and the same move is evaluated again.
 * accept_dev (nullable): dev, n_moves bytes, 1 = accepted.  stats_host
 * (nullable) receives the run's statistics. */
bhmc_status bhmc_mc_run(bhmc_tree* tree, int32_t replica, uint64_t seed, uint64_t move0,
                        int64_t n_moves, double step, uint8_t* accept_dev, bhmc_stats* stats_host);

/* Advance every replica by n_sweeps sweeps of N_r moves each, all replicas in
 * one persistent launch per sweep (one workgroup per replica at a time,
 * largest replica first).  Replica r's sweeps use move indices continuing
 * from its own move counter (0 after build), so replica r alone through
 * bhmc_mc_run with the same seed gives the same chain.  use_graph = 1 captures
 * one sweep in a hipGraph and replays it.  Replicas that stop before a move
 * that would overflow a leaf index array are rebuilt together after the sweep
 * and finish it in one more persistent launch, so every sweep ends with every
 * replica at the end of its sweep.  stats_host (nullable): R entries. */
bhmc_status bhmc_batch_sweep(bhmc_tree* tree, uint64_t seed, int32_t n_sweeps, double step,
                             int32_t use_graph, bhmc_stats* stats_host);

/* Autotuner of the Metropolis kernel's launch shape and traversal tile.
 * Times trial_moves moves (at most N_r) of every replica with each candidate
 * (shape s, tile j): shape 0: 512-thread workgroups, one per CU; 1:
 * 256-thread workgroups, one per CU; 2: 256-thread workgroups, two per CU;
 * tile 0: one trial move per traversal (two targets); 1: half the most moves
 * per round the order allows; 2: the most (see bhmc_set_moves_per_round;
 * tiles 1 and 2 only when every replica has N_0 = 0 and no line images, and tile 1 only when it
 * is above one move).  Every replica is rebuilt from its built positions
 * after each trial, and the fastest candidate is kept for the handle's later
 * bhmc_mc_run and bhmc_batch_sweep calls (replacing the moves per round set
 * before).  Needs the replicas as built (no moves run yet; EINVAL otherwise)
 * and leaves them exactly as built.  choice (nullable, host): 3 s + j of the
 * candidate kept; ms_host (nullable, host, 9 floats): trial time of
 * candidate 3 s + j (0 if not tried: a one-replica handle tries shapes 0 and
 * 1 only).  The chain of a replica depends on the candidate only through the
 * rounding of its energy sums. */
bhmc_status bhmc_batch_autotune(bhmc_tree* tree, uint64_t seed, double step, int32_t trial_moves,
                                int32_t* choice, float* ms_host);

/* Set the Metropolis kernel's launch shape (0, 1 or 2 as for
 * bhmc_batch_autotune) directly, e.g. to the shape the autotuner chose on
 * another handle of the same workload (with bhmc_set_moves_per_round for its
 * tile).  EINVAL for another value. */
bhmc_status bhmc_set_launch_shape(bhmc_tree* tree, int32_t shape);

/* Gradient of the treecode energy E of bhmc_energy for replica `replica`,
 * exact for the interaction lists its traversal makes (each far pair term
 * q_t q_j sum_n T_n(r_A - r_t) (r_j - r_A)^n of eq. 3.3 and each near pair
 * q_t q_j / |r_t - r_j| is differentiated in both its points and charges; the
 * images are mapped back to their ions by the chain rule through
 * q_K = gamma a q / |r|, r_K = a^2 r / |r|^2, line images through t_m r_K and
 * -sigma w_m q_K).  It uses the replica's current
 * moments, which equal a fresh evaluation from the current positions up to
 * rounding (bhmc_rebuild refreshes them); nothing of the traversal is stored.
 * Outputs: dEdr_dev (dev, 3n values, x y z per ion), dEdq_dev (dev, n
 * values); E_host (nullable) receives E, equal to bhmc_energy's up to the
 * rounding of its sums (about 1e-15 relative).  The
 * far-field source side is summed with device atomics, so the gradient can
 * differ between calls by rounding.  The library keeps a workspace of
 * about 8 (ncell * round4(C(p+3,3)) + 4.5 nsrc + 5 n) bytes per handle. */
bhmc_status bhmc_energy_grad(bhmc_tree* tree, int32_t replica, double* dEdr_dev, double* dEdq_dev,
                             double* E_host);

/* Trial moves evaluated together by bhmc_mc_run and bhmc_batch_sweep (and the
 * autotuner).  moves = 1: one move at a time (evaluate, decide, commit).
 * moves = 0 (the default) or > 1: rounds of up to that many consecutive moves
 * of distinct ions (at most 8 for p <= 8, 2 above), evaluated in
 * one traversal of the tree as it stands at the start of the round and then
 * decided and committed in order, each energy change corrected exactly for the
 * moves accepted before it in the round (Sec. 3.2 with N_0 = 0: the
 * traversal's decisions depend only on geometry and occupancy, so an accepted
 * move changes a later move's potentials only through its own contributions).
 * The chain -- accept stream, positions, statistics -- is the same as with one
 * move at a time, up to the rounding of the energy sums.  Handles with a replica
 * with N_0 > 0 or with line images always run one move at a time.  effective
 * (nullable, host) receives the moves per round the handle will use. */
bhmc_status bhmc_set_moves_per_round(bhmc_tree* tree, int32_t moves, int32_t* effective);

/* Phase timers of the batched Metropolis kernel, present only in a library
 * built with phase timers (python -m paper_1305_1825_amd.build --phase-timers):
 * ticks of the device's constant clock summed over every round run on this
 * handle's expansion order -- set-up, traversal levels, corrected moments and
 * scan, far cells, near leaves, hard cores below far cells, path descents,
 * corrections, decisions, leaf index arrays, moments -- then the number of
 * rounds and of moves, the level loop's chunks, frontier entries, empty
 * entries, far and near list entries, and the ticks the root-path descents
 * and the commit prefetch spend inside the level loop.  ticks: host, n values; count (nullable, host) receives
 * the number of counters (0 for a library built without timers, which then
 * writes nothing).  reset = 1 clears them after reading. */
bhmc_status bhmc_phase_ticks(bhmc_tree* tree, uint64_t* ticks, int32_t n, int32_t reset, int32_t* count);

/* Frontier capacity of the breadth-first MAC traversals (Sec. 3.2).  A level
 * keeps up to lds_entries frontier entries on chip (64..4096; 4096 after
 * build).  With allow_spill = 1 (the default) a level that outgrows them
 * continues in HBM regions the library allocates the first time this happens
 * (per handle, 8 B per cell of the largest replica per workgroup region, one
 * region per workgroup of a launch), and the call that stopped runs again; a
 * traversal then never fails for lack of frontier space, so theta = 0 (the
 * direct sum) works at any size.  With allow_spill = 0 such a call returns
 * BHMC_ESTACK instead.  The results do not depend on where the frontier lives. */
bhmc_status bhmc_set_frontier_capacity(bhmc_tree* tree, int32_t lds_entries, int32_t allow_spill);

/* Current ion positions and charges of a replica (dev outputs, n each). */
bhmc_status bhmc_get_state(bhmc_tree* tree, int32_t replica, double* x, double* y, double* z,
                           double* q);

/* Recompute a replica's moments (eq. 3.3) from the current members of its
 * leaves, on the tree as it stands (no change of cells or leaf index
 * arrays): P2M at the leaves, then M2M up the tree.  Accepted moves repair the
 * moments incrementally (Sec. 3.3); this replaces them by a fresh sum, which
 * differs from the repaired one only by rounding. */
bhmc_status bhmc_refresh_moments(bhmc_tree* tree, int32_t replica);

/* Rebuild a replica's tree from its current positions. */
bhmc_status bhmc_rebuild(bhmc_tree* tree, int32_t replica);

/* Introspection for checking (host outputs, any of them nullable):
 *   bhmc_get_sorted: keys (nsrc u64) in ascending order and the source index
 *     of each (nsrc i32), ties by source index, as built.
 *   bhmc_get_cells: per cell (ncell): level (i32), smallest key of the cell
 *     (u64), current count N_A (i32), link (i32: first child >= 0, or -1-leaf
 *     for a leaf), geometry (4 f64: centre x y z, half side h), moments
 *     (nterms f64 per cell, graded multi-index order s = 0..p, n1 = s..0,
 *     n2 = s-n1..0).  Cells are numbered level by level, children of a cell
 *     consecutive in digit order 4 x + 2 y + z.
 *   bhmc_get_leaves: per leaf (nleaf): cell (i32), slot base (i32), capacity
 *     (i32), build range begin/end in the sorted order (i32).
 *   bhmc_get_slots: the pool (pool i32): source index in each slot; leaf l
 *     holds slots base[l] .. base[l] + count of its cell - 1. */
bhmc_status bhmc_get_sorted(bhmc_tree* tree, int32_t replica, uint64_t* keys, int32_t* index);
bhmc_status bhmc_get_cells(bhmc_tree* tree, int32_t replica, int32_t* level, uint64_t* kmin,
                           int32_t* count, int32_t* link, double* geo, double* moments);
bhmc_status bhmc_get_leaves(bhmc_tree* tree, int32_t replica, int32_t* cell, int32_t* base,
                            int32_t* cap, int32_t* begin, int32_t* end);
bhmc_status bhmc_get_slots(bhmc_tree* tree, int32_t replica, int32_t* slots);

/* Message for the last non-OK status on this thread. */
const char* bhmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BHMC_H */
