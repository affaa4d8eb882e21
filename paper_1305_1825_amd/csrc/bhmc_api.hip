// Host side of the C ABI declared in include/bhmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "bhmc.h"
#include "bhmc_dev.hpp"
#include "bhmc_internal.hpp"

namespace bhmc {

const EvalOps* eval_ops_p0(); const EvalOps* eval_ops_p1(); const EvalOps* eval_ops_p2();
const EvalOps* eval_ops_p3(); const EvalOps* eval_ops_p4(); const EvalOps* eval_ops_p5();
const EvalOps* eval_ops_p6(); const EvalOps* eval_ops_p7(); const EvalOps* eval_ops_p8();
const EvalOps* eval_ops_p9(); const EvalOps* eval_ops_p10();

const EvalOps* eval_ops(int p) {
    switch (p) {
        case 0: return eval_ops_p0(); case 1: return eval_ops_p1(); case 2: return eval_ops_p2();
        case 3: return eval_ops_p3(); case 4: return eval_ops_p4(); case 5: return eval_ops_p5();
        case 6: return eval_ops_p6(); case 7: return eval_ops_p7(); case 8: return eval_ops_p8();
        case 9: return eval_ops_p9(); case 10: return eval_ops_p10();
        default: return nullptr;
    }
}

// ------------------------------------------------------------ utility kernels
__global__ void k_sweep_prep(Rep* reps, int R, int* queue, const long long* add) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x)
        reps[r].move_end += add[r];
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
}

__global__ void k_reset_queue(int* queue) { *queue = 0; }

__global__ void k_unpack(const double4* src, int n, double* x, double* y, double* z, double* q) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double4 v = src[i];
        if (x) x[i] = v.x;
        if (y) y[i] = v.y;
        if (z) z[i] = v.z;
        if (q) q[i] = v.w;
    }
}

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated sum of v[0..n) times scale into *out (one workgroup).
__global__ void __launch_bounds__(1024) k_sum(const double* v, int n, double scale, double* out) {
    __shared__ double ss[1024], cc[1024];
    double s = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        double t, e;
        two_sum(s, v[k], t, e);
        s = t; c += e;
    }
    ss[threadIdx.x] = s; cc[threadIdx.x] = c;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double t, e;
            two_sum(ss[threadIdx.x], ss[threadIdx.x + w], t, e);
            ss[threadIdx.x] = t;
            cc[threadIdx.x] += cc[threadIdx.x + w] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * (ss[0] + cc[0]);
}

void launch_sweep_prep(hipStream_t s, Rep* reps, int R, int* queue, const long long* add) {
    hipLaunchKernelGGL(k_sweep_prep, dim3((R + 255) / 256), dim3(256), 0, s, reps, R, queue, add);
}
void launch_reset_queue(hipStream_t s, int* queue) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, s, queue);
}
void launch_sum(hipStream_t s, const double* v, int n, double scale, double* out) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, v, n, scale, out);
}

}  // namespace bhmc

using bhmc::Rep;

// ------------------------------------------------------------ fixed scratch memory
// Per-ion energy terms of bhmc_energy_noalloc live in this file-scope device
// array instead of library allocations.  In host code the name stands for a
// host-side shadow, not a device address: kernels and copies only ever get the
// address hipGetSymbolAddress returns, resolved once per device when the first
// handle is created on it (each device holds its own copy of the array).
constexpr int kScratchDoubles = 1 << 19;  // 4 MiB: energy terms of up to 524,288 ions
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on the current device (null on failure).
static double* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_dev[dev] = (double*)ptr;
    }
    return g_scratch_dev[dev];
}

// ------------------------------------------------------------ handle
struct bhmc_tree {
    int R = 0, p = 0, nterms = 0, mstride = 0;
    hipStream_t stream = nullptr;
    std::vector<bhmc_params> params;
    Rep* host = nullptr;             // pinned mirror of the descriptor table
    char* pin = nullptr;             // pinned staging for every other host<->device copy
    size_t pin_bytes = 0;
    Rep* reps = nullptr;             // device descriptor table
    std::vector<void*> arena1, arena2;
    const bhmc::EvalOps* ops = nullptr;
    int* queue = nullptr;
    int* list_all = nullptr;         // replicas, largest first
    int* list_one = nullptr;         // scratch list of one replica
    int* list_rest = nullptr;        // replicas a sweep left unfinished
    std::vector<int> order;          // replicas, largest first (host copy of list_all)
    long long* sweep_add = nullptr;  // n_r per replica
    int* build_list = nullptr;       // replicas of a build (at most R)
    long long* build_off = nullptr;  // their first ion in the caller's arrays
    bhmc::MoveIO* io = nullptr;
    double* eterm = nullptr; int eterm_n = 0;
    char* gwork = nullptr; size_t gwork_bytes = 0;  // gradient workspace
    int* wide_buf = nullptr;         // grid-wide build of one large replica: sort histograms, level counts
    double* scalar = nullptr;
    double* scratch = nullptr;       // device address of the fixed scratch array on the handle's device
    // HBM frontier regions, allocated the first time a traversal level outgrows its LDS capacity
    uint32_t* spill = nullptr;
    int spill_regions = 0;
    long long spill_words = 0;       // 32-bit words per region
    int fcap = 4096;                 // frontier entries a level keeps in LDS
    int allow_spill = 1;
    bool energy_bounded = false;     // energy / gradient launches keep their grid within the regions
    int moves_per_round = 0;         // 0: as many as the order allows; 1: the move-by-move kernel
    bool rounds_ok = true;           // the rounds kernel needs N_0 = 0 and no line images on every replica
    bool has_lines = false;          // some replica has line images
    int mc_grid = 1;
    int mc_wide = 1;                 // one replica: the 512-thread Metropolis kernel
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;  // capture needs a stream other than the null stream
    uint64_t graph_seed = 0; double graph_step = 0.0; bool graph_ok = false;
};

static thread_local std::string g_err;

static bhmc_status fail(bhmc_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static bhmc_status fail(bhmc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? BHMC_ENOMEM : BHMC_EHIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                               \
    } while (0)

extern "C" const char* bhmc_last_error(void) { return g_err.c_str(); }

// The M-point Gauss rule for the weight t^(sigma - 1) on [0, 1], the line image of the
// multiple-image model: by Golub and Welsch, the nodes are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the polynomials orthogonal for that weight (the
// Jacobi polynomials P^(0, sigma - 1) moved to [0, 1]) and the weights are the squared
// first components of its unit eigenvectors times the weight's integral 1 / sigma.  The
// eigenproblem (at most 8 x 8) is solved by cyclic Jacobi rotations.  Nodes descending,
// nodes and weights rounded to multiples of 2^-40 (far below the rule's own error).
static bool line_rule(double sigma, int M, double* t, double* w) {
    if (M < 1 || M > 8 || !(sigma >= 0.5 && sigma <= 1.0)) return false;
    const double b = sigma - 1.0;
    double A[8][8] = {}, V[8][8] = {};
    for (int k = 0; k < M; ++k) {
        // recurrence coefficients of the monic Jacobi (0, b) polynomials on [-1, 1]
        const double c = 2.0 * k + b;
        const double diag = k == 0 ? b / (b + 2.0) : (b * b) / (c * (c + 2.0));
        A[k][k] = 0.5 * (1.0 + diag);  // t = (1 + x) / 2
        if (k + 1 < M) {
            const double j = k + 1.0, c1 = 2.0 * j + b;
            const double beta = 4.0 * j * j * (j + b) * (j + b) / (c1 * c1 * (c1 + 1.0) * (c1 - 1.0));
            A[k][k + 1] = A[k + 1][k] = 0.5 * std::sqrt(beta);
        }
        V[k][k] = 1.0;
    }
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < M; ++i) {
            diag += A[i][i] * A[i][i];
            for (int j = i + 1; j < M; ++j) off += A[i][j] * A[i][j];
        }
        if (off <= 1e-34 * diag) break;
        for (int p = 0; p < M; ++p)
            for (int q = p + 1; q < M; ++q) {
                if (A[p][q] == 0.0) continue;
                // the rotation in the (p, q) plane that zeroes A[p][q]
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double tn = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(tn * tn + 1.0), sn = tn * cs;
                for (int k = 0; k < M; ++k) {  // columns p and q
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < M; ++k) {  // rows p and q
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < M; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    int order[8];
    for (int k = 0; k < M; ++k) order[k] = k;
    std::sort(order, order + M, [&](int i, int j) { return A[i][i] > A[j][j]; });
    for (int m = 0; m < M; ++m) {
        const int k = order[m];
        t[m] = std::ldexp(std::nearbyint(std::ldexp(A[k][k], 40)), -40);
        w[m] = std::ldexp(std::nearbyint(std::ldexp(V[0][k] * V[0][k] / sigma, 40)), -40);
    }
    return true;
}

static bhmc_status check_params(const bhmc_params& P, int64_t n) {
    if (n < 1 || n > (1 << 22)) return fail(BHMC_EINVAL, "n = %lld out of range [1, 2^22]", (long long)n);
    if (!(P.theta >= 0.0 && P.theta < 1.0)) return fail(BHMC_EINVAL, "theta must lie in [0, 1)");
    if (P.p < 0 || P.p > bhmc::kPMax) return fail(BHMC_EINVAL, "p must lie in [0, %d]", bhmc::kPMax);
    if (P.leaf_cap < 0 || P.n0 < 0) return fail(BHMC_EINVAL, "leaf_cap and n0 must be >= 0");
    if (P.max_depth < 0 || P.max_depth > bhmc::kMaxDepth) return fail(BHMC_EINVAL, "max_depth must lie in [0, 21]");
    if (P.slot_slack < 1 || P.slot_slack > 1024) return fail(BHMC_EINVAL, "slot_slack must lie in [1, 1024]");
    if (P.leaf_cap > (1 << 23)) return fail(BHMC_EINVAL, "leaf_cap must be <= 2^23");
    if (!(P.box_side > 0.0) || !std::isfinite(P.box_side)) return fail(BHMC_EINVAL, "box_side must be > 0");
    if (P.geom != 0 && P.geom != 1) return fail(BHMC_EINVAL, "geom must be 0 or 1");
    if (P.images && P.geom != 1) return fail(BHMC_EINVAL, "images need the spherical geometry");
    if (P.geom == 1 && !(P.r_min >= 0.0 && P.r_min < P.r_max)) return fail(BHMC_EINVAL, "need 0 <= r_min < r_max");
    if (P.geom == 1) {
        // every point of the shell (|r| < r_max) must lie in the root cube [lo, lo + side)^3
        for (int d = 0; d < 3; ++d)
            if (!(P.box_lo[d] <= -P.r_max && P.box_lo[d] + P.box_side >= P.r_max))
                return fail(BHMC_EINVAL, "the root cube must contain the shell |r| < r_max");
    }
    if (P.images && !(P.a > 0.0 && P.a <= P.r_min && P.eps_in > 0.0 && P.eps_out >= 0.0))
        return fail(BHMC_EINVAL, "images need 0 < a <= r_min and eps_in > 0");
    if (!(P.hard_core >= 0.0) || !(P.l_B >= 0.0)) return fail(BHMC_EINVAL, "hard_core and l_B must be >= 0");
    if (P.far_fp32 != 0 && P.far_fp32 != 1) return fail(BHMC_EINVAL, "far_fp32 must be 0 or 1");
    if (P.line_images < 0 || P.line_images > 8) return fail(BHMC_EINVAL, "line_images must lie in [0, 8]");
    if (P.line_images > 0) {
        const double sigma = P.eps_out / (P.eps_in + P.eps_out);
        if (!P.images) return fail(BHMC_EINVAL, "line images need images = 1");
        if (P.n0 != 0) return fail(BHMC_EINVAL, "line images need N_0 = 0");
        if (!(sigma >= 0.5 && sigma <= 1.0)) return fail(BHMC_EINVAL, "line images need eps_in <= eps_out");
        if ((2 + P.line_images) * n > (1 << 23)) return fail(BHMC_EINVAL, "too many sources with line images");
    }
    return BHMC_OK;
}

static void fill_rep(Rep& r, const bhmc_params& P, int64_t n) {
    memset(&r, 0, sizeof(Rep));
    for (int d = 0; d < 3; ++d) { r.lo[d] = P.box_lo[d]; r.hi[d] = P.box_lo[d] + P.box_side; }
    r.side = P.box_side;
    r.scale = 2097152.0 / P.box_side;
    r.theta2 = P.theta * P.theta;
    r.l_B = P.l_B;
    r.a = P.a;
    r.a2 = P.a * P.a;
    r.gamma = (P.eps_out + P.eps_in) != 0.0 ? (P.eps_out - P.eps_in) / (P.eps_out + P.eps_in) : 0.0;
    r.Qc = P.geom == 1 ? P.Q_center : 0.0;
    r.rmin2 = P.r_min * P.r_min;
    r.rmax2 = P.r_max * P.r_max;
    r.tau2 = P.hard_core * P.hard_core;
    {
        const double reach = P.hard_core + 1e-12 * P.box_side;
        r.reach2 = reach * reach;
    }
    r.geom = P.geom; r.images = P.images; r.leaf_cap = P.leaf_cap; r.n0 = P.n0;
    r.far32 = P.far_fp32 ? 1 : 0;
    r.max_depth = P.max_depth; r.slack = P.slot_slack;
    r.n = (int)n;
    r.nline = 0;
    if (P.images && P.line_images > 0) {
        const double sigma = P.eps_out / (P.eps_in + P.eps_out);
        double w[8];
        if (line_rule(sigma, P.line_images, r.line_t, w)) {
            r.nline = P.line_images;
            for (int m = 0; m < r.nline; ++m) r.line_c[m] = -sigma * w[m];
        }
    }
    r.nsrc = P.images ? (2 + r.nline) * (int)n : (int)n;
    r.fcap = 4096;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Every host<->device copy goes through pinned memory the library allocated
// itself (hipHostMalloc); caller or stack memory is never handed to HIP.
static bhmc_status ensure_pin(bhmc_tree* t, size_t bytes) {
    if (bytes <= t->pin_bytes) return BHMC_OK;
    size_t want = std::max(bytes, (size_t)1 << 16);
    if (t->pin) { hipHostFree(t->pin); t->pin = nullptr; t->pin_bytes = 0; }
    HIP_TRY(hipHostMalloc((void**)&t->pin, want, hipHostMallocDefault));
    t->pin_bytes = want;
    return BHMC_OK;
}

static bhmc_status d2h(bhmc_tree* t, void* dst, const void* src_dev, size_t bytes) {
    if (!bytes) return BHMC_OK;
    bhmc_status st = ensure_pin(t, bytes);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(t->pin, src_dev, bytes, hipMemcpyDeviceToHost, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));
    memcpy(dst, t->pin, bytes);
    return BHMC_OK;
}

static bhmc_status h2d(bhmc_tree* t, void* dst_dev, const void* src, size_t bytes) {
    if (!bytes) return BHMC_OK;
    bhmc_status st = ensure_pin(t, bytes);
    if (st) return st;
    memcpy(t->pin, src, bytes);
    HIP_TRY(hipMemcpyAsync(dst_dev, t->pin, bytes, hipMemcpyHostToDevice, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));  // the staging buffer is reused at once
    return BHMC_OK;
}

struct Carver {
    char* base; size_t off = 0;
    template <class T> T* take(size_t count) {
        T* p = (T*)(base + off);
        off = align_up(off + sizeof(T) * (count ? count : 1));
        return p;
    }
};

static size_t phase1_bytes(int nsrc) {
    size_t b = 0;
    b += align_up(32 * (size_t)nsrc); b += 3 * align_up(8 * (size_t)nsrc); b += 2 * align_up(4 * (size_t)nsrc);
    return b;
}

static bhmc_status alloc_phase1(bhmc_tree* t, int r) {
    Rep& h = t->host[r];
    if (t->arena1[r]) { hipFree(t->arena1[r]); t->arena1[r] = nullptr; }
    HIP_TRY(hipMalloc(&t->arena1[r], phase1_bytes(h.nsrc)));
    Carver c{(char*)t->arena1[r]};
    h.src = c.take<double4>(h.nsrc);
    h.keys = c.take<uint64_t>(h.nsrc); h.ktmp = c.take<uint64_t>(h.nsrc);
    h.perm = c.take<int>(h.nsrc); h.ptmp = c.take<int>(h.nsrc);
    h.track = c.take<int2>(h.nsrc);
    if (c.off > phase1_bytes(h.nsrc)) return fail(BHMC_EINTERNAL, "source arena carved past its allocation");
    return BHMC_OK;
}

static bhmc_status alloc_phase2(bhmc_tree* t, int r) {
    Rep& h = t->host[r];
    if (t->arena2[r]) { hipFree(t->arena2[r]); t->arena2[r] = nullptr; }
    const size_t nc = h.ncell, nl = h.nleaf, np = h.pool;
    size_t b = align_up(32 * nc) + align_up(16 * nc) + 4 * align_up(4 * nc) + align_up(8 * nc) +
               align_up(8 * nc * (size_t)t->mstride) + 3 * align_up(4 * nl) + align_up(32 * np) +
               align_up(4 * np) + (h.far32 ? align_up(4 * nc * (size_t)t->mstride) : 0);
    HIP_TRY(hipMalloc(&t->arena2[r], b));
    Carver c{(char*)t->arena2[r]};
    const size_t cap_bytes = b;
    h.cgeo = c.take<double4>(nc);
    h.cm = c.take<int4>(nc); h.cparent = c.take<int>(nc);
    h.clevel = c.take<int>(nc); h.cbegin = c.take<int>(nc); h.cend = c.take<int>(nc);
    h.ckey = c.take<uint64_t>(nc);
    h.M = c.take<double>(nc * (size_t)t->mstride);
    h.lcell = c.take<int>(nl); h.lbase = c.take<int>(nl); h.lcap = c.take<int>(nl);
    h.pool4 = c.take<double4>(np); h.pidx = c.take<int>(np);
    h.M32 = h.far32 ? c.take<float>(nc * (size_t)t->mstride) : nullptr;
    if (c.off > cap_bytes) return fail(BHMC_EINTERNAL, "tree arena carved past its allocation");
    return BHMC_OK;
}

static bhmc_status upload(bhmc_tree* t) {
    HIP_TRY(hipMemcpyAsync(t->reps, t->host, sizeof(Rep) * t->R, hipMemcpyHostToDevice, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));  // the host mirror may change right after
    return BHMC_OK;
}
static bhmc_status download(bhmc_tree* t) {
    HIP_TRY(hipMemcpyAsync(t->host, t->reps, sizeof(Rep) * t->R, hipMemcpyDeviceToHost, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));
    return BHMC_OK;
}

// Frontier regions in HBM for every workgroup that may need one: one per workgroup of the
// Metropolis launch and of a bounded energy / gradient launch.  A region holds the two levels a
// traversal keeps at once of its widest possible frontier: 4 targets x every cell (energy,
// 32-bit entries), or every cell with a 32-bit cell and a 64-bit mask word (gradient).  Sized
// for the replicas' current cell counts; returns whether it had to grow.
static bhmc_status ensure_spill(bhmc_tree* t, bool* grown) {
    *grown = false;
    long long maxc = 1;
    for (int r = 0; r < t->R; ++r) maxc = std::max<long long>(maxc, t->host[r].ncell);
    const long long words = (8 * maxc + 16 + 63) & ~63ll;
    int dev = 0, ncu = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int regions = std::max(std::max(512, 2 * ncu), t->mc_grid);
    if (t->spill && words <= t->spill_words && regions <= t->spill_regions) return BHMC_OK;
    if (t->spill) { hipFree(t->spill); t->spill = nullptr; t->spill_words = 0; t->spill_regions = 0; }
    HIP_TRY(hipMalloc(&t->spill, sizeof(uint32_t) * (size_t)words * regions));
    t->spill_words = words;
    t->spill_regions = regions;
    for (int r = 0; r < t->R; ++r) {
        t->host[r].spill = t->spill;
        t->host[r].spill_words = words;
        t->host[r].spill_regions = regions;
    }
    *grown = true;
    return BHMC_OK;
}

// After a traversal stopped with detail `detail`: true if it stopped because a level outgrew
// the LDS frontier and HBM regions (now allocated or grown) let it run again.
static bool retry_with_spill(bhmc_tree* t, int detail, bhmc_status* st) {
    *st = BHMC_OK;
    if (detail != bhmc::kErrFrontier || !t->allow_spill) return false;
    bool grown = false;
    if ((*st = ensure_spill(t, &grown))) return false;
    return grown;
}

static const char* status_name(int s) {
    switch (s) {
        case -1: return "a non-finite coordinate or charge";
        case -2: return "an ion outside the confinement, or a source outside the root cube";
        case -5: return "inconsistent tree sizes";
        case -8: return "a device-side index check failed while filling the leaf arrays";
        default: return "error";
    }
}

// Build (or rebuild) the replicas in `list`.  x == nullptr rebuilds from the
// replicas' own current ions.
static bhmc_status build_list(bhmc_tree* t, const std::vector<int>& list, const double* x,
                              const double* y, const double* z, const double* q,
                              const std::vector<long long>& ion_off) {
    const int nr = (int)list.size();
    if (nr < 1 || nr > t->R) return fail(BHMC_EINTERNAL, "build of %d replicas", nr);
    int* dlist = t->build_list;       // per-handle buffers: no allocation per build
    long long* doff = t->build_off;
    bhmc_status st = h2d(t, dlist, list.data(), sizeof(int) * nr);
    if (st) return st;
    if (x && (st = h2d(t, doff, ion_off.data(), sizeof(long long) * nr))) return st;
    for (int r : list)
        if (!t->host[r].src && (st = alloc_phase1(t, r))) return st;
    st = upload(t);
    if (st) return st;
    const int nsrc0 = t->host[list[0]].nsrc;
    if (nr == 1 && nsrc0 >= bhmc::kWideBuildMin) {
        // one large replica: sources, sort and count over a grid of workgroups (same results)
        if (!t->wide_buf) {
            const size_t bytes = sizeof(int) * (256 * bhmc::kSortGridMax + bhmc::kCountLevels + 64);
            HIP_TRY(hipMalloc(&t->wide_buf, bytes));
            HIP_TRY(hipMemsetAsync(t->wide_buf, 0, bytes, t->stream));
        }
        bhmc::launch_sources_wide(t->stream, t->reps, list[0], t->host[list[0]].n, x, y, z, q, x ? doff : nullptr,
                                  t->wide_buf + 256 * bhmc::kSortGridMax + bhmc::kCountLevels);
        bhmc::launch_sort_wide(t->stream, t->reps, list[0], nsrc0, t->wide_buf);
        bhmc::launch_count_wide(t->stream, t->reps, list[0], nsrc0, t->wide_buf + 256 * bhmc::kSortGridMax);
    } else {
        bhmc::launch_sources(t->stream, nr, t->reps, dlist, x, y, z, q, x ? doff : nullptr);
        bhmc::launch_sort(t->stream, nr, t->reps, dlist);
        bhmc::launch_count(t->stream, nr, t->reps, dlist);
    }
    HIP_TRY(hipGetLastError());
    if ((st = download(t))) return st;
    for (int r : list) {
        Rep& h = t->host[r];
        if (h.status == -4)
            return fail(BHMC_EINVAL, "replica %d: leaf index arrays of slot_slack * (sources + leaves * leaf_cap) "
                        "slots exceed 2^31", r);
        if (h.status) return fail(h.status == -1 ? BHMC_EINVAL : BHMC_EOUTSIDE, "replica %d: %s", r, status_name(h.status));
        if (h.ncell >= (1 << 24)) return fail(BHMC_EINVAL, "replica %d: %d cells exceed 2^24", r, h.ncell);
    }
    for (int r : list) if ((st = alloc_phase2(t, r))) return st;
    if ((st = upload(t))) return st;
    bhmc::launch_topology(t->stream, nr, t->reps, dlist);
    if (nr == 1 && nsrc0 >= bhmc::kWideBuildMin)
        bhmc::launch_leaves_wide(t->stream, t->reps, dlist, list[0], t->host[list[0]].nleaf);
    else
        bhmc::launch_leaves(t->stream, nr, t->reps, dlist);
    HIP_TRY(hipGetLastError());
    if ((st = download(t))) return st;  // cells per level size the moment launches
    for (int r : list)
        if (t->host[r].status) return fail(BHMC_EHIP, "replica %d: %s", r, status_name(t->host[r].status));
    bhmc::launch_moments(t->stream, nr, t->reps, dlist, t->nterms, t->mstride, t->host, list.data());
    HIP_TRY(hipGetLastError());
    if ((st = download(t))) return st;
    for (int r : list)
        if (t->host[r].status) return fail(BHMC_EHIP, "replica %d: %s", r, status_name(t->host[r].status));
    return BHMC_OK;
}

static void destroy(bhmc_tree* t) {
    if (!t) return;
    if (t->gexec) hipGraphExecDestroy(t->gexec);
    if (t->graph) hipGraphDestroy(t->graph);
    if (t->graph_stream) hipStreamDestroy(t->graph_stream);
    for (void* p : t->arena1) if (p) hipFree(p);
    for (void* p : t->arena2) if (p) hipFree(p);
    hipFree(t->reps); hipFree(t->queue); hipFree(t->list_all); hipFree(t->list_one); hipFree(t->list_rest);
    hipFree(t->sweep_add); hipFree(t->build_list); hipFree(t->build_off); hipFree(t->io); hipFree(t->eterm); hipFree(t->scalar); hipFree(t->gwork);
    hipFree(t->spill); hipFree(t->wide_buf);
    if (t->host) hipHostFree(t->host);
    if (t->pin) hipHostFree(t->pin);
    delete t;
}

static bhmc_status create(const bhmc_params* params, int32_t R, const int64_t* n_per, const double* x,
                          const double* y, const double* z, const double* q, void* stream,
                          bhmc_tree** out) {
    if (!out) return fail(BHMC_EINVAL, "out is null");
    *out = nullptr;
    if (R < 1 || !params || !n_per) return fail(BHMC_EINVAL, "need R >= 1 replicas");
    if (!x || !y || !z || !q) return fail(BHMC_EINVAL, "null input array");
    for (int r = 0; r < R; ++r) {
        bhmc_status st = check_params(params[r], n_per[r]);
        if (st) return st;
        if (params[r].p != params[0].p) return fail(BHMC_EINVAL, "all replicas must share p");
    }
    bhmc_tree* t = new bhmc_tree();
    t->R = R;
    t->p = params[0].p;
    t->nterms = bhmc::nterms_of(t->p);
    t->mstride = bhmc::mstride_of(t->p);
    t->stream = (hipStream_t)stream;
    t->params.assign(params, params + R);
    if (hipHostMalloc((void**)&t->host, sizeof(Rep) * R, hipHostMallocDefault) != hipSuccess) {
        delete t;
        return fail(BHMC_ENOMEM, "pinned descriptor mirror");
    }
    t->arena1.assign(R, nullptr);
    t->arena2.assign(R, nullptr);
    t->ops = bhmc::eval_ops(t->p);
    for (int r = 0; r < R; ++r) {
        if (params[r].line_images > 0) t->has_lines = true;
        if (params[r].n0 != 0 || params[r].line_images > 0) t->rounds_ok = false;
    }
    std::vector<long long> off(R);
    long long acc = 0;
    for (int r = 0; r < R; ++r) { fill_rep(t->host[r], params[r], n_per[r]); off[r] = acc; acc += n_per[r]; }
    auto bail = [&](bhmc_status st) { destroy(t); return st; };
    if (hipMalloc(&t->reps, sizeof(Rep) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "descriptor table"));
    if (hipMalloc(&t->queue, sizeof(int)) != hipSuccess) return bail(fail(BHMC_ENOMEM, "queue"));
    if (hipMalloc(&t->list_all, sizeof(int) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "list"));
    if (hipMalloc(&t->list_one, sizeof(int)) != hipSuccess) return bail(fail(BHMC_ENOMEM, "list"));
    if (hipMalloc(&t->list_rest, sizeof(int) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "list"));
    if (hipMalloc(&t->sweep_add, sizeof(long long) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "sweep"));
    if (hipMalloc(&t->build_list, sizeof(int) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "build list"));
    if (hipMalloc(&t->build_off, sizeof(long long) * R) != hipSuccess) return bail(fail(BHMC_ENOMEM, "build list"));
    if (hipMalloc(&t->io, sizeof(bhmc::MoveIO)) != hipSuccess) return bail(fail(BHMC_ENOMEM, "io"));
    if (hipMalloc(&t->scalar, sizeof(double) * 4) != hipSuccess) return bail(fail(BHMC_ENOMEM, "scalar"));
    if (ensure_pin(t, 1 << 16) != BHMC_OK) return bail(BHMC_ENOMEM);
    if (bhmc::upload_build_tables(t->p, t->pin) != hipSuccess) return bail(fail(BHMC_EHIP, "constant tables"));
    std::vector<int> list(R);
    std::iota(list.begin(), list.end(), 0);
    bhmc_status st = build_list(t, list, x, y, z, q, off);
    if (st) return bail(st);
    // largest replica first in the sweep queue
    std::vector<int> order(R);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n_per[a] > n_per[b]; });
    t->order = order;
    std::vector<long long> add(n_per, n_per + R);
    if ((st = h2d(t, t->list_all, order.data(), sizeof(int) * R)) ||
        (st = h2d(t, t->sweep_add, add.data(), sizeof(long long) * R)))
        return bail(st);
    int dev = 0, ncu = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    t->scratch = scratch_address(dev);
    if (!t->scratch) return bail(fail(BHMC_EHIP, "cannot resolve the scratch array on device %d", dev));
    // one replica: one wide workgroup; replicas: two 256-thread workgroups per CU.  A handle
    // always runs the same kernel, so a replica's chain does not depend on how it is advanced.
    t->mc_wide = R == 1 ? 1 : 0;
    t->mc_grid = R == 1 ? 1 : std::max(1, std::min(R, 2 * (ncu > 0 ? ncu : 256)));
    *out = t;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_build(const bhmc_params* params, int64_t n, const double* x, const double* y,
                                  const double* z, const double* q, void* hip_stream, bhmc_tree** out) {
    return create(params, 1, &n, x, y, z, q, hip_stream, out);
}

extern "C" bhmc_status bhmc_batch_create(const bhmc_params* params, int32_t R, const int64_t* n_per_replica,
                                         const double* x, const double* y, const double* z, const double* q,
                                         void* hip_stream, bhmc_tree** out) {
    return create(params, R, n_per_replica, x, y, z, q, hip_stream, out);
}

extern "C" void bhmc_free(bhmc_tree* tree) {
    if (tree) hipStreamSynchronize(tree->stream);
    destroy(tree);
}

extern "C" int32_t bhmc_replicas(const bhmc_tree* tree) { return tree ? tree->R : 0; }

static bhmc_status check_rep(bhmc_tree* t, int32_t r) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    if (r < 0 || r >= t->R) return fail(BHMC_EINVAL, "replica %d out of range", r);
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_info_get(bhmc_tree* tree, int32_t replica, bhmc_info* info) {
    bhmc_status st = check_rep(tree, replica);
    if (st) return st;
    if (!info) return fail(BHMC_EINVAL, "null info");
    const Rep& h = tree->host[replica];
    info->n = h.n; info->nsrc = h.nsrc; info->ncell = h.ncell; info->nleaf = h.nleaf;
    info->nterms = tree->nterms; info->depth = h.depth; info->pool = h.pool;
    return BHMC_OK;
}

static bhmc_status rebuild_one(bhmc_tree* t, int r) {
    bhmc_status st = download(t);  // keep the kernel-side counters of every replica
    if (st) return st;
    std::vector<int> list{r};
    return build_list(t, list, nullptr, nullptr, nullptr, nullptr, {});
}

extern "C" bhmc_status bhmc_refresh_moments(bhmc_tree* t, int32_t replica) {
    bhmc_status st = check_rep(t, replica);
    if (st) return st;
    if ((st = h2d(t, t->list_one, &replica, sizeof(int)))) return st;
    bhmc::launch_moments(t->stream, 1, t->reps, t->list_one, t->nterms, t->mstride, t->host, &replica);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(t->stream));
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_rebuild(bhmc_tree* tree, int32_t replica) {
    bhmc_status st = check_rep(tree, replica);
    if (st) return st;
    return rebuild_one(tree, replica);
}

static bhmc_status ensure_eterm(bhmc_tree* t, int n) {
    if (t->eterm_n < n) {
        hipFree(t->eterm);
        t->eterm = nullptr;
        t->eterm_n = 0;
        HIP_TRY(hipMalloc(&t->eterm, sizeof(double) * n));
        t->eterm_n = n;
    }
    return BHMC_OK;
}

// Sum of the per-ion energy terms; a NaN there marks a failed traversal.  *again: the
// traversal ran out of LDS frontier and should run again with HBM regions (now allocated).
static bhmc_status finish_energy(bhmc_tree* t, int r, int n, double* E_host, const char* what, bool* again) {
    *again = false;
    bhmc::launch_sum(t->stream, t->eterm, n, t->host[r].l_B, t->scalar);
    HIP_TRY(hipGetLastError());
    double E = 0.0;
    bhmc_status st = d2h(t, &E, t->scalar, sizeof(double));
    if (st) return st;
    if (std::isnan(E)) {
        if ((st = download(t))) return st;
        const int d = t->host[r].err_detail;
        if (retry_with_spill(t, d, &st) || (d == bhmc::kErrFrontier && t->spill && !t->energy_bounded)) {
            t->host[r].err_detail = 0;
            t->energy_bounded = true;
            if ((st = upload(t))) return st;
            *again = true;
            return BHMC_OK;
        }
        if (st) return st;
        if (d > 1 && d != bhmc::kErrFrontier)
            return fail(BHMC_EINTERNAL, "device index check %d failed in the %s traversal", d, what);
        return fail(BHMC_ESTACK, "a traversal list outgrew its capacity");
    }
    if (E_host) *E_host = E;
    return BHMC_OK;
}

static int energy_grid_bound(const bhmc_tree* t) { return t->energy_bounded && t->spill ? t->spill_regions : 0; }

extern "C" bhmc_status bhmc_energy(bhmc_tree* t, int32_t replica, double* E_host, double* phi_dev) {
    bhmc_status st = check_rep(t, replica);
    if (st) return st;
    const int n = t->host[replica].n;
    if ((st = ensure_eterm(t, n))) return st;
    for (;;) {
        t->ops->energy(t->stream, t->reps, replica, n, phi_dev, t->eterm, energy_grid_bound(t), t->host[replica].nline);
        HIP_TRY(hipGetLastError());
        bool again = false;
        if ((st = finish_energy(t, replica, n, E_host, "energy", &again)) || !again) return st;
    }
}

// The energy of bhmc_energy with its per-ion terms in the fixed scratch array and
// the total written to device memory: nothing is allocated and nothing waits
// for the device, so the call can be captured in a graph.
extern "C" bhmc_status bhmc_energy_noalloc(bhmc_tree* t, int32_t replica, double* E_dev, double* phi_dev) {
    bhmc_status st = check_rep(t, replica);
    if (st) return st;
    if (!E_dev) return fail(BHMC_EINVAL, "null energy output");
    const int n = t->host[replica].n;
    if (n > kScratchDoubles)
        return fail(BHMC_EINVAL, "replica %d has %d ions; the allocation-free energy takes at most %d", replica, n,
                    kScratchDoubles);
    if (!t->scratch) return fail(BHMC_EHIP, "scratch array not resolved");
    t->ops->energy(t->stream, t->reps, replica, n, phi_dev, t->scratch, energy_grid_bound(t), t->host[replica].nline);
    bhmc::launch_sum(t->stream, t->scratch, n, t->host[replica].l_B, E_dev);
    HIP_TRY(hipGetLastError());
    return BHMC_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" bhmc_status bhmc_energy_grad(bhmc_tree* t, int32_t replica, double* dEdr_dev, double* dEdq_dev,
                                        double* E_host) {
    bhmc_status st = check_rep(t, replica);
    if (st) return st;
    if (!dEdr_dev || !dEdq_dev) return fail(BHMC_EINVAL, "null gradient output");
    if (!t->ops->grad) return fail(BHMC_EINVAL, "gradient not available for p = %d", t->p);
    const Rep& h = t->host[replica];
    const int n = h.n;
    if ((st = ensure_eterm(t, n))) return st;
    const size_t lb = align256(sizeof(double) * (size_t)h.ncell * t->mstride);
    const size_t gb = align256(sizeof(double) * 4 * (size_t)h.nsrc);
    const size_t tb = align256(sizeof(double) * 4 * (size_t)n);
    const size_t ob = align256(sizeof(int) * ((size_t)h.nsrc + 1));
    const size_t ib = align256(sizeof(int) * (size_t)n);
    const size_t need = lb + gb + tb + ob + 2 * ib;
    if (t->gwork_bytes < need) {
        hipFree(t->gwork);
        t->gwork = nullptr;
        t->gwork_bytes = 0;
        HIP_TRY(hipMalloc(&t->gwork, need));
        t->gwork_bytes = need;
    }
    bhmc::GradWork w;
    w.L = (double*)t->gwork;
    w.G = (double4*)(t->gwork + lb);
    w.Gt = (double4*)(t->gwork + lb + gb);
    w.rank = (int*)(t->gwork + lb + gb + tb);
    w.islot = (int*)(t->gwork + lb + gb + tb + ob);
    w.fcell = (int*)(t->gwork + lb + gb + tb + ob + ib);
    w.ncell = h.ncell; w.nleaf = h.nleaf; w.nsrc = h.nsrc; w.n = n; w.nline = h.nline;
    for (;;) {
        t->ops->grad(t->stream, t->reps, replica, w, dEdr_dev, dEdq_dev, t->eterm, energy_grid_bound(t));
        HIP_TRY(hipGetLastError());
        bool again = false;
        if ((st = finish_energy(t, replica, n, E_host, "gradient", &again)) || !again) return st;
    }
}

static bhmc_status run_move(bhmc_tree* t, int64_t i, const double* r_new, int mode, bhmc::MoveIO& io) {
    bhmc_status st = check_rep(t, 0);
    if (st) return st;
    if (i < 0 || i >= t->host[0].n) return fail(BHMC_EINVAL, "ion index %lld out of range", (long long)i);
    if (!r_new || !std::isfinite(r_new[0]) || !std::isfinite(r_new[1]) || !std::isfinite(r_new[2]))
        return fail(BHMC_EINVAL, "r_new must be three finite values");
    memset(&io, 0, sizeof(io));
    io.i = (int)i;
    io.rn[0] = r_new[0]; io.rn[1] = r_new[1]; io.rn[2] = r_new[2];
    io.mode = mode;
    const bhmc::MoveIO io_in = io;
    for (;;) {
        io = io_in;
        if ((st = h2d(t, t->io, &io, sizeof(io)))) return st;
        t->ops->move(t->stream, t->reps, 0, t->io, t->has_lines ? 1 : 0);
        HIP_TRY(hipGetLastError());
        if ((st = d2h(t, &io, t->io, sizeof(io)))) return st;
        if (io.status != -7) break;
        if ((st = download(t))) return st;
        if (retry_with_spill(t, t->host[0].err_detail, &st)) {
            t->host[0].err_detail = 0;
            if ((st = upload(t))) return st;
            continue;
        }
        if (st) return st;
        return fail(BHMC_ESTACK, "a traversal list outgrew its capacity");
    }
    if (io.status == -8) {
        bhmc_status s2 = download(t);
        if (s2) return s2;
        return fail(BHMC_EINTERNAL, "device index check %d failed", t->host[0].err_detail);
    }
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_delta_energy(bhmc_tree* tree, int64_t i, const double* r_new, double* dE_host,
                                         int32_t* reason_host) {
    bhmc::MoveIO io;
    if (!tree) return fail(BHMC_EINVAL, "null tree");
    bhmc_status st = run_move(tree, i, r_new, 0, io);
    if (st) return st;
    if (dE_host) *dE_host = io.reason ? HUGE_VAL : io.dE;
    if (reason_host) *reason_host = io.reason;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_commit_move(bhmc_tree* tree, int64_t i, const double* r_new) {
    bhmc::MoveIO io;
    if (!tree) return fail(BHMC_EINVAL, "null tree");
    bhmc_status st = run_move(tree, i, r_new, 1, io);
    if (st) return st;
    if (io.reason == 1) return fail(BHMC_EINVAL, "the move leaves the confinement");
    if (io.reason == 2) return fail(BHMC_EOVERLAP, "the move overlaps a hard core");
    if (io.status == -6) return fail(BHMC_ECAPACITY, "a leaf index array is full; rebuild first");
    return BHMC_OK;
}

// Moves per round the handle's Metropolis launches take (1 = the move-by-move kernel).
static int rounds_of(const bhmc_tree* t) {
    if (t->moves_per_round == 1 || !t->rounds_ok) return 1;
    const int cap = t->ops->moves_per_round;
    return t->moves_per_round > 1 && t->moves_per_round < cap ? t->moves_per_round : cap;
}

static void launch_mc(bhmc_tree* t, hipStream_t s, bhmc::McArgs a, int grid, int wide) {
    const int bm = rounds_of(t);
    a.lines = t->has_lines ? 1 : 0;
    if (bm <= 1) {
        t->ops->mc(s, t->reps, a, grid, wide);
    } else {
        a.bm = bm;
        t->ops->mcb(s, t->reps, a, grid, wide);
    }
}

static bhmc_status run_replica_until_done(bhmc_tree* t, int r, const bhmc::McArgs& base, long long* rebuilds) {
    long long last_stop = -1;
    for (;;) {
        bhmc::McArgs a = base;
        a.list = t->list_one;
        a.nlist = 1;
        bhmc_status st0 = h2d(t, t->list_one, &r, sizeof(int));
        if (st0) return st0;
        bhmc::launch_reset_queue(t->stream, t->queue);
        launch_mc(t, t->stream, a, 1, t->mc_wide);
        HIP_TRY(hipGetLastError());
        bhmc_status st = download(t);
        if (st) return st;
        const Rep& h = t->host[r];
        if (h.mc_status == -7) {
            if (retry_with_spill(t, h.err_detail, &st)) {
                // nothing of the stopped move was committed: run it again with HBM frontier regions
                t->host[r].mc_status = 0;
                t->host[r].err_detail = 0;
                if ((st = upload(t))) return st;
                continue;
            }
            if (st) return st;
            return fail(BHMC_ESTACK, "replica %d: a traversal list outgrew its capacity", r);
        }
        if (h.mc_status == -8)
            return fail(BHMC_EINTERNAL, "replica %d: device index check %d failed at move %lld", r, h.err_detail, h.move_next);
        if (h.mc_status == -6) {
            // a fresh tree leaves two spare slots in every leaf, so the same
            // move cannot overflow twice in a row
            if (h.move_next == last_stop)
                return fail(BHMC_ECAPACITY, "replica %d: move %lld overflows a fresh tree", r, h.move_next);
            last_stop = h.move_next;
            if ((st = rebuild_one(t, r))) return st;
            ++*rebuilds;
            continue;
        }
        return BHMC_OK;
    }
}

extern "C" bhmc_status bhmc_mc_run(bhmc_tree* t, int32_t replica, uint64_t seed, uint64_t move0,
                                   int64_t n_moves, double step, uint8_t* accept_dev, bhmc_stats* stats_host) {
    bhmc_status st = check_rep(t, replica);
    if (st) return st;
    if (n_moves < 0 || !std::isfinite(step)) return fail(BHMC_EINVAL, "bad n_moves or step");
    if ((st = download(t))) return st;
    Rep& h = t->host[replica];
    h.move_next = (long long)move0;
    h.move_end = (long long)(move0 + n_moves);
    h.mc_status = 0;
    for (int k = 0; k < 6; ++k) h.stats[k] = 0;
    if ((st = upload(t))) return st;
    bhmc::McArgs a{};
    a.seed = seed;
    a.step = step;
    a.queue = t->queue;
    a.accept = accept_dev;
    a.move_base = (long long)move0;
    long long rebuilds = 0;
    if ((st = run_replica_until_done(t, replica, a, &rebuilds))) return st;
    if (stats_host) {
        const Rep& g = t->host[replica];
        stats_host->moves = g.stats[0]; stats_host->accepted = g.stats[1];
        stats_host->rejected_wall = g.stats[2]; stats_host->rejected_overlap = g.stats[3];
        stats_host->rejected_metropolis = g.stats[4]; stats_host->rebuilds = rebuilds;
    }
    return BHMC_OK;
}

// Replicas that a sweep left unfinished stopped before a move that would
// overflow a leaf index array.  All of them are rebuilt in one build launch and
// the rest of their moves run in one persistent launch over just those
// replicas (largest first), until every replica has finished the sweep.
static bhmc_status finish_sweep(bhmc_tree* t, const bhmc::McArgs& base, std::vector<long long>& rebuilds,
                                std::vector<long long>& last_stop) {
    for (;;) {
        bhmc_status st = download(t);
        if (st) return st;
        std::vector<int> stalled, rest;
        bool respill = false;
        for (int r : t->order) {
            Rep& h = t->host[r];
            if (h.mc_status == -7) {
                bool grown = false;
                if (h.err_detail == bhmc::kErrFrontier && t->allow_spill && !respill) {
                    if ((st = ensure_spill(t, &grown))) return st;
                    respill = grown;
                }
                if (!respill) return fail(BHMC_ESTACK, "replica %d: a traversal list outgrew its capacity", r);
                h.mc_status = 0;  // its stopped move runs again with HBM frontier regions
                h.err_detail = 0;
            }
            if (h.mc_status == -8)
                return fail(BHMC_EINTERNAL, "replica %d: device index check %d failed at move %lld", r, h.err_detail,
                            h.move_next);
            if (h.mc_status == -6) {
                // a fresh tree leaves two spare slots in every leaf, so the same
                // move cannot overflow twice in a row
                if (h.move_next == last_stop[r])
                    return fail(BHMC_ECAPACITY, "replica %d: move %lld overflows a fresh tree", r, h.move_next);
                last_stop[r] = h.move_next;
                stalled.push_back(r);
            }
            if (h.mc_status == -6 || h.move_next < h.move_end) rest.push_back(r);
        }
        if (rest.empty()) return BHMC_OK;
        if (!stalled.empty()) {
            if ((st = build_list(t, stalled, nullptr, nullptr, nullptr, nullptr, {}))) return st;
            for (int r : stalled) ++rebuilds[r];
        }
        for (int r : rest) t->host[r].mc_status = 0;
        (void)respill;
        if ((st = upload(t))) return st;
        if ((st = h2d(t, t->list_rest, rest.data(), sizeof(int) * rest.size()))) return st;
        bhmc::McArgs a = base;
        a.list = t->list_rest;
        a.nlist = (int)rest.size();
        bhmc::launch_reset_queue(t->stream, t->queue);
        launch_mc(t, t->stream, a, std::min((int)rest.size(), t->mc_grid), t->mc_wide);
        HIP_TRY(hipGetLastError());
    }
}

extern "C" bhmc_status bhmc_batch_sweep(bhmc_tree* t, uint64_t seed, int32_t n_sweeps, double step,
                                        int32_t use_graph, bhmc_stats* stats_host) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    if (n_sweeps < 0 || !std::isfinite(step)) return fail(BHMC_EINVAL, "bad n_sweeps or step");
    bhmc_status st = download(t);
    if (st) return st;
    for (int r = 0; r < t->R; ++r) {
        t->host[r].move_next = t->host[r].move_end;  // sweeps continue from the chain's end
        t->host[r].mc_status = 0;
        for (int k = 0; k < 6; ++k) t->host[r].stats[k] = 0;
    }
    if ((st = upload(t))) return st;
    bhmc::McArgs a{};
    a.seed = seed;
    a.step = step;
    a.list = t->list_all;
    a.nlist = t->R;
    a.queue = t->queue;
    std::vector<long long> rebuilds(t->R, 0), last_stop(t->R, -1);
    hipStream_t gs = t->stream;
    if (use_graph) {
        if (!gs) {
            if (!t->graph_stream) HIP_TRY(hipStreamCreateWithFlags(&t->graph_stream, hipStreamNonBlocking));
            gs = t->graph_stream;
            HIP_TRY(hipDeviceSynchronize());
        }
        if (!t->graph_ok || t->graph_seed != seed || t->graph_step != step) {
            if (t->gexec) { hipGraphExecDestroy(t->gexec); t->gexec = nullptr; }
            if (t->graph) { hipGraphDestroy(t->graph); t->graph = nullptr; }
            HIP_TRY(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
            bhmc::launch_sweep_prep(gs, t->reps, t->R, t->queue, t->sweep_add);
            launch_mc(t, gs, a, t->mc_grid, t->mc_wide);
            HIP_TRY(hipStreamEndCapture(gs, &t->graph));
            HIP_TRY(hipGraphInstantiate(&t->gexec, t->graph, nullptr, nullptr, 0));
            t->graph_ok = true; t->graph_seed = seed; t->graph_step = step;
        }
    }
    for (int s = 0; s < n_sweeps; ++s) {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(t->gexec, gs));
            if (gs != t->stream) HIP_TRY(hipStreamSynchronize(gs));
        } else {
            bhmc::launch_sweep_prep(t->stream, t->reps, t->R, t->queue, t->sweep_add);
            launch_mc(t, t->stream, a, t->mc_grid, t->mc_wide);
        }
        HIP_TRY(hipGetLastError());
        if ((st = finish_sweep(t, a, rebuilds, last_stop))) return st;
    }
    if (stats_host) {
        for (int r = 0; r < t->R; ++r) {
            const Rep& g = t->host[r];
            bhmc_stats& s = stats_host[r];
            s.moves = g.stats[0]; s.accepted = g.stats[1]; s.rejected_wall = g.stats[2];
            s.rejected_overlap = g.stats[3]; s.rejected_metropolis = g.stats[4]; s.rebuilds = rebuilds[r];
        }
    }
    return BHMC_OK;
}

// Launch shapes the replica autotuner tries: workgroup width (512 or 256
// threads per traversal) and workgroups per CU (one, or two of 256 threads);
// with each, up to three traversal tiles (trial moves per round).
struct LaunchShape { int wide, per_cu; };
static const LaunchShape kShapes[] = {{1, 1}, {0, 1}, {0, 2}};
constexpr int kAutotuneTiles = 3;

extern "C" bhmc_status bhmc_batch_autotune(bhmc_tree* t, uint64_t seed, double step, int32_t trial_moves,
                                           int32_t* choice, float* ms_out) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    if (trial_moves < 1 || !std::isfinite(step)) return fail(BHMC_EINVAL, "bad trial_moves or step");
    bhmc_status st = download(t);
    if (st) return st;
    for (int r = 0; r < t->R; ++r)
        if (t->host[r].move_end != 0 || t->host[r].stats[0] != 0)
            return fail(BHMC_EINVAL, "autotune needs replicas as built (replica %d has moved)", r);
    int dev = 0, ncu = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
    // the built positions, to rebuild every replica exactly as built after each trial
    std::vector<long long> off(t->R);
    long long ntot = 0;
    for (int r = 0; r < t->R; ++r) { off[r] = ntot; ntot += t->host[r].n; }
    double* saved = nullptr;
    HIP_TRY(hipMalloc(&saved, sizeof(double) * 4 * (size_t)ntot));
    struct Free { double* p; ~Free() { hipFree(p); } } guard{saved};
    double *sx = saved, *sy = saved + ntot, *sz = saved + 2 * ntot, *sq = saved + 3 * ntot;
    for (int r = 0; r < t->R; ++r) {
        const Rep& h = t->host[r];
        hipLaunchKernelGGL(bhmc::k_unpack, dim3(std::max(1, std::min(1024, (h.n + 255) / 256))), dim3(256), 0,
                           t->stream, (const double4*)h.src, h.n, sx + off[r], sy + off[r], sz + off[r], sq + off[r]);
    }
    HIP_TRY(hipGetLastError());
    std::vector<int> all(t->R);
    std::iota(all.begin(), all.end(), 0);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.0f;
    int best = -1;
    const int nshape = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
    // moves per round (targets per shared traversal): one at a time, half the most, the most
    const int cap = t->rounds_ok ? t->ops->moves_per_round : 1;
    const int tiles[kAutotuneTiles] = {1, cap / 2 > 1 ? cap / 2 : 0, cap > 1 ? cap : 0};
    const int saved_mpr = t->moves_per_round;
    if (ms_out)
        for (int k = 0; k < nshape * kAutotuneTiles; ++k) ms_out[k] = 0.0f;
    for (int k = 0; k < nshape * kAutotuneTiles && st == BHMC_OK; ++k) {
        const LaunchShape sh = kShapes[k / kAutotuneTiles];
        if (t->R == 1 && sh.per_cu > 1) continue;  // one workgroup in all: two per CU is the same shape
        if (tiles[k % kAutotuneTiles] == 0) continue;
        t->moves_per_round = tiles[k % kAutotuneTiles];
        for (int r = 0; r < t->R; ++r) {
            Rep& h = t->host[r];
            h.move_next = 0;
            h.move_end = std::min<long long>(trial_moves, h.n);
            h.mc_status = 0;
        }
        if ((st = upload(t))) break;
        bhmc::McArgs a{};
        a.seed = seed; a.step = step; a.list = t->list_all; a.nlist = t->R; a.queue = t->queue;
        bhmc::launch_reset_queue(t->stream, t->queue);
        const int grid = std::max(1, std::min(t->R, sh.per_cu * ncu));
        if (hipEventRecord(e0, t->stream) != hipSuccess) { st = fail(BHMC_EHIP, "event"); break; }
        launch_mc(t, t->stream, a, grid, sh.wide);
        if (hipEventRecord(e1, t->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = fail(BHMC_EHIP, "trial launch failed");
            break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms_out) ms_out[k] = ms;
        if (best < 0 || ms < best_ms) { best = k; best_ms = ms; }
        // back to the replicas as built
        if ((st = download(t))) break;
        if ((st = build_list(t, all, sx, sy, sz, sq, off))) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    t->moves_per_round = saved_mpr;
    if (st) return st;
    if ((st = download(t))) return st;
    for (int r = 0; r < t->R; ++r) {
        Rep& h = t->host[r];
        h.move_next = h.move_end = 0;
        h.mc_status = 0;
        h.err_detail = 0;
        for (int q = 0; q < 6; ++q) h.stats[q] = 0;
    }
    if ((st = upload(t))) return st;
    t->mc_wide = kShapes[best / kAutotuneTiles].wide;
    t->mc_grid = std::max(1, std::min(t->R, kShapes[best / kAutotuneTiles].per_cu * ncu));
    t->moves_per_round = tiles[best % kAutotuneTiles];
    t->graph_ok = false;
    if (choice) *choice = best;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_set_launch_shape(bhmc_tree* t, int32_t shape) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    const int nshape = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
    if (shape < 0 || shape >= nshape) return fail(BHMC_EINVAL, "launch shape %d out of range", shape);
    int dev = 0, ncu = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
    t->mc_wide = kShapes[shape].wide;
    t->mc_grid = std::max(1, std::min(t->R, kShapes[shape].per_cu * ncu));
    t->graph_ok = false;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_set_moves_per_round(bhmc_tree* t, int32_t moves, int32_t* effective) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    if (moves < 0) return fail(BHMC_EINVAL, "moves per round must be >= 0");
    t->moves_per_round = moves;
    t->graph_ok = false;
    if (effective) *effective = rounds_of(t);
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_phase_ticks(bhmc_tree* t, uint64_t* ticks, int32_t n, int32_t reset, int32_t* count) {
    if (!t || !ticks || n < 0) return fail(BHMC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(t->stream));
    const int k = t->ops->phases((unsigned long long*)ticks, n, reset);
    if (k < 0) return fail(BHMC_EHIP, "reading the phase timers failed");
    if (count) *count = k;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_set_frontier_capacity(bhmc_tree* t, int32_t lds_entries, int32_t allow_spill) {
    if (!t) return fail(BHMC_EINVAL, "null tree");
    if (lds_entries < 64 || lds_entries > 4096) return fail(BHMC_EINVAL, "lds_entries must lie in [64, 4096]");
    bhmc_status st = download(t);
    if (st) return st;
    t->fcap = lds_entries;
    t->allow_spill = allow_spill ? 1 : 0;
    for (int r = 0; r < t->R; ++r) t->host[r].fcap = lds_entries;
    return upload(t);
}

extern "C" bhmc_status bhmc_get_state(bhmc_tree* t, int32_t r, double* x, double* y, double* z, double* q) {
    bhmc_status st = check_rep(t, r);
    if (st) return st;
    const Rep& h = t->host[r];
    hipLaunchKernelGGL(bhmc::k_unpack, dim3(std::max(1, std::min(1024, (h.n + 255) / 256))), dim3(256), 0,
                       t->stream, (const double4*)h.src, h.n, x, y, z, q);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(t->stream));
    return BHMC_OK;
}

// ---- introspection: host outputs, staged through pinned memory
extern "C" bhmc_status bhmc_get_sorted(bhmc_tree* t, int32_t r, uint64_t* keys, int32_t* index) {
    bhmc_status st = check_rep(t, r);
    if (st) return st;
    const Rep& h = t->host[r];
    if (keys && (st = d2h(t, keys, h.keys, 8 * (size_t)h.nsrc))) return st;
    if (index && (st = d2h(t, index, h.perm, 4 * (size_t)h.nsrc))) return st;
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_get_cells(bhmc_tree* t, int32_t r, int32_t* level, uint64_t* kmin, int32_t* count,
                                      int32_t* link, double* geo, double* moments) {
    bhmc_status st = check_rep(t, r);
    if (st) return st;
    const Rep& h = t->host[r];
    const size_t nc = h.ncell;
    if (level && (st = d2h(t, level, h.clevel, 4 * nc))) return st;
    if (kmin && (st = d2h(t, kmin, h.ckey, 8 * nc))) return st;
    if (count || link) {
        std::vector<int4> cm(nc);
        if ((st = d2h(t, cm.data(), h.cm, 16 * nc))) return st;
        for (size_t c = 0; c < nc; ++c) {
            if (count) count[c] = cm[c].x;
            if (link) link[c] = cm[c].y;
        }
    }
    if (geo && (st = d2h(t, geo, h.cgeo, 32 * nc))) return st;
    if (moments) {
        std::vector<double> rows(nc * (size_t)t->mstride);
        if ((st = d2h(t, rows.data(), h.M, sizeof(double) * rows.size()))) return st;
        for (size_t c = 0; c < nc; ++c)
            memcpy(moments + c * t->nterms, rows.data() + c * t->mstride, sizeof(double) * t->nterms);
    }
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_get_leaves(bhmc_tree* t, int32_t r, int32_t* cell, int32_t* base, int32_t* cap,
                                       int32_t* begin, int32_t* end) {
    bhmc_status st = check_rep(t, r);
    if (st) return st;
    const Rep& h = t->host[r];
    std::vector<int> lc(h.nleaf), cb(h.ncell), ce(h.ncell);
    if ((st = d2h(t, lc.data(), h.lcell, 4 * (size_t)h.nleaf))) return st;
    if ((st = d2h(t, cb.data(), h.cbegin, 4 * (size_t)h.ncell))) return st;
    if ((st = d2h(t, ce.data(), h.cend, 4 * (size_t)h.ncell))) return st;
    if (cell) memcpy(cell, lc.data(), 4 * (size_t)h.nleaf);
    if (base && (st = d2h(t, base, h.lbase, 4 * (size_t)h.nleaf))) return st;
    if (cap && (st = d2h(t, cap, h.lcap, 4 * (size_t)h.nleaf))) return st;
    for (int l = 0; l < h.nleaf; ++l) {
        if (begin) begin[l] = cb[lc[l]];
        if (end) end[l] = ce[lc[l]];
    }
    return BHMC_OK;
}

extern "C" bhmc_status bhmc_get_slots(bhmc_tree* t, int32_t r, int32_t* slots) {
    bhmc_status st = check_rep(t, r);
    if (st) return st;
    const Rep& h = t->host[r];
    if (slots && (st = d2h(t, slots, h.pidx, 4 * (size_t)h.pool))) return st;
    return BHMC_OK;
}
