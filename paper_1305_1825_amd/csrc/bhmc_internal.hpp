// Declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bhmc {

struct Rep;

constexpr int kMaxTerms = 364;  // (p+1)(p+2)(p+3)/6 at p = 11 (gradient needs order p + 1)

inline int nterms_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
inline int mstride_of(int p) { return (nterms_of(p) + 3) & ~3; }  // 32-byte aligned rows

// Arguments of one Monte Carlo launch.
struct McArgs {
    uint64_t seed;
    double step;
    const int* list;      // replica ids to run, in queue order
    int nlist;
    int* queue;           // work-queue counter (reset before the launch)
    uint8_t* accept;      // per-move accept bits of a single-replica run, or null
    long long move_base;  // move index of accept[0]
    long long* sweep_add; // per replica moves added to move_end by the sweep prep kernel
    int bm;               // batched kernel: moves per round (0 = as many as the order allows)
    int lines;            // 1: a replica has line images (the move kernel with their steps)
};

// One externally specified move (delta_energy / commit_move).
struct MoveIO {
    int i;
    double rn[3];
    int mode;             // 0: evaluate only; 1: evaluate and commit unless rejected
    double dE;
    int reason;
    int status;
};

// ---- build (bhmc_build.hip)
hipError_t upload_build_tables(int p, void* pinned);  // pinned: >= 16 KiB of hipHostMalloc memory
void launch_sources(hipStream_t s, int nrep, Rep* reps, const int* list, const double* x,
                    const double* y, const double* z, const double* q, const long long* ion_off);
void launch_sort(hipStream_t s, int nrep, Rep* reps, const int* list);
void launch_count(hipStream_t s, int nrep, Rep* reps, const int* list);
// One large replica over a grid of workgroups, with the same results: the sort
// uses hist (256 * kSortGridMax ints), the count cnt (kCountLevels ints) and the
// sources flag (one int), both zero before the call and zero again after it.
constexpr int kSortGridMax = 256;
constexpr int kCountLevels = 64;
constexpr int kWideBuildMin = 32768;  // sources from which a single-replica build goes wide
void launch_sources_wide(hipStream_t s, Rep* reps, int r, int n, const double* x, const double* y,
                         const double* z, const double* q, const long long* ion_off, int* flag);
void launch_sort_wide(hipStream_t s, Rep* reps, int r, int nsrc, int* hist);
void launch_count_wide(hipStream_t s, Rep* reps, int r, int nsrc, int* cnt);
void launch_leaves_wide(hipStream_t s, Rep* reps, const int* list, int r, int nleaf);
void launch_topology(hipStream_t s, int nrep, Rep* reps, const int* list);
void launch_leaves(hipStream_t s, int nrep, Rep* reps, const int* list);
// host / host_list: the host mirror of the descriptors (sizes and levels as counted) and the replicas
void launch_moments(hipStream_t s, int nrep, Rep* reps, const int* list, int nterms, int mstride,
                    const Rep* host, const int* host_list);

// Workspace of one gradient evaluation (device memory, library-owned).
struct GradWork {
    double* L;            // adjoint coefficients, ncell rows of mstride
    double4* G;           // per source: dE/dx, dE/dy, dE/dz, dE/dq through its source role
    double4* Gt;          // per ion: the same through its target role
    int* rank;            // per sorted source: ions before it (nsrc + 1)
    int* islot;           // per ion rank: its current slot (n)
    int* fcell;           // per ion: the far cell holding its own image in its traversal, or -1 (n)
    int ncell, nleaf, nsrc, n;
    int nline;            // line images per ion (multiple-image model), 0 without
};

// ---- evaluation (bhmc_eval.hip, one translation unit per expansion order)
struct EvalOps {
    // wide = 1: 512-thread workgroups (one chain); 0: 256-thread workgroups, two per CU (replicas)
    void (*mc)(hipStream_t s, Rep* reps, const McArgs& a, int grid, int wide);
    // the same chains with several trial moves per round (N_0 = 0 only)
    void (*mcb)(hipStream_t s, Rep* reps, const McArgs& a, int grid, int wide);
    int moves_per_round;  // the most the batched kernel takes per round at this order
    void (*move)(hipStream_t s, Rep* reps, int r, MoveIO* io_dev, int lines);
    // max_grid > 0 bounds the number of workgroups (each then takes several target groups), so that
    // every workgroup has an HBM frontier region
    // nline > 0: the replica has line images (multiple-image model), corrected after the traversal
    void (*energy)(hipStream_t s, Rep* reps, int r, int n, double* phi, double* eterm, int max_grid, int nline);
    void (*grad)(hipStream_t s, Rep* reps, int r, const GradWork& w, double* dEdr, double* dEdq,
                 double* eterm, int max_grid);
    // phase timers of the batched Metropolis kernel: number of counters, 0 without timers
    int (*phases)(unsigned long long* out, int n, int reset);
};
const EvalOps* eval_ops(int p);

// ---- small utility kernels (bhmc_api.hip)
void launch_sweep_prep(hipStream_t s, Rep* reps, int R, int* queue, const long long* add);
void launch_reset_queue(hipStream_t s, int* queue);
void launch_sum(hipStream_t s, const double* v, int n, double scale, double* out);

}  // namespace bhmc
