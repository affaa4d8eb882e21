// Treecode evaluation kernels for one expansion order p (compiled once per p
// with -DBHMC_P=p, so every recurrence index below is a compile-time constant
// and the Taylor coefficients live in registers).
//
// Traversal (Sec. 3.2).  A workgroup evaluates the potential at a few targets
// at once.  The MAC traversal runs breadth first: the frontier of one level
// sits in LDS, every lane classifies one (cell, target) entry, and a block
// scan hands out slots in the far list, the near list and the next frontier,
// so the order of every list, and therefore every sum, is deterministic.
// Far cells are evaluated lane-per-cell with the recurrence of eq. 3.4 fused
// into the dot product with the moments of eq. 3.3; near leaves are flattened
// into (leaf, slot) pairs read from the leaf-ordered pool, so the lanes of a
// wave read consecutive slots.
//
// Exclusion.  The mover i and its image are taken out of the source set: a
// frontier entry carries two bits telling whether its cell holds them (the
// bits follow the digits of their keys down the tree).  At most one far cell
// per (target, excluded source) can hold one of them, so the corrected
// moments M - q (r - c)^n of those cells are formed in LDS.
#include "bhmc_dev.hpp"
#include "bhmc_internal.hpp"

#include <algorithm>

#ifndef BHMC_P
#error "compile once per expansion order with -DBHMC_P=<p>"
#endif

#define BHMC_CAT2(a, b) a##b
#define BHMC_CAT(a, b) BHMC_CAT2(a, b)
#define BHMC_NS BHMC_CAT(eval_p, BHMC_P)

namespace bhmc {
namespace BHMC_NS {

constexpr int P = BHMC_P;
constexpr int NTERM = (P + 1) * (P + 2) * (P + 3) / 6;
constexpr int MSTR = (NTERM + 3) & ~3;  // moment row stride (32-byte rows)

// ------------------------------------------------------------ index tables
constexpr int cmindex(int n1, int n2, int n3) {
    int s = n1 + n2 + n3;
    return s * (s + 1) * (s + 2) / 6 + (s - n1) * (s - n1 + 1) / 2 + (s - n1 - n2);
}

struct TEnt { int n1, n2, n3, s, x1, y1, z1, x2, y2, z2; };
template <int N>
struct TTab { TEnt e[N]; };

// entries of every multi-index up to order PP, in the graded order above
template <int PP>
constexpr TTab<(PP + 1) * (PP + 2) * (PP + 3) / 6> make_tab() {
    TTab<(PP + 1) * (PP + 2) * (PP + 3) / 6> t{};
    int k = 0;
    for (int s = 0; s <= PP; ++s)
        for (int n1 = s; n1 >= 0; --n1)
            for (int n2 = s - n1; n2 >= 0; --n2) {
                const int n3 = s - n1 - n2;
                TEnt e{};
                e.n1 = n1; e.n2 = n2; e.n3 = n3; e.s = s;
                e.x1 = n1 >= 1 ? cmindex(n1 - 1, n2, n3) : -1;
                e.y1 = n2 >= 1 ? cmindex(n1, n2 - 1, n3) : -1;
                e.z1 = n3 >= 1 ? cmindex(n1, n2, n3 - 1) : -1;
                e.x2 = n1 >= 2 ? cmindex(n1 - 2, n2, n3) : -1;
                e.y2 = n2 >= 2 ? cmindex(n1, n2 - 2, n3) : -1;
                e.z2 = n3 >= 2 ? cmindex(n1, n2, n3 - 2) : -1;
                t.e[k++] = e;
            }
    return t;
}
constexpr auto TT = make_tab<P>();
// one order more for the field, dT_n/dR_k = (n_k + 1) T_{n + e_k}; the first
// NTERM entries coincide with TT
constexpr int NTERM1 = (P + 2) * (P + 3) * (P + 4) / 6;
constexpr auto TT1 = make_tab<P + 1>();

struct MiTab { int v[3 * NTERM]; };
constexpr MiTab make_mi() {
    MiTab m{};
    for (int k = 0; k < NTERM; ++k) { m.v[3 * k] = TT.e[k].n1; m.v[3 * k + 1] = TT.e[k].n2; m.v[3 * k + 2] = TT.e[k].n3; }
    return m;
}
__constant__ MiTab c_mi = make_mi();

// (n1, n2, n3) of term k packed as n1 | n2 << 8 | n3 << 16; workgroups keep a
// copy of this table in LDS, so runtime term indices read it there
__device__ __forceinline__ uint32_t mi_code(int k) {
    return (uint32_t)c_mi.v[3 * k] | ((uint32_t)c_mi.v[3 * k + 1] << 8) | ((uint32_t)c_mi.v[3 * k + 2] << 16);
}

// d^n by repeated multiplication (x, then y, then z), as the moments are built
__device__ __forceinline__ double mono(uint32_t code, double dx, double dy, double dz) {
    const int n1 = (int)(code & 255u), n2 = (int)((code >> 8) & 255u), n3 = (int)(code >> 16);
    double v = 1.0;
    for (int e = 0; e < n1; ++e) v *= dx;
    for (int e = 0; e < n2; ++e) v *= dy;
    for (int e = 0; e < n3; ++e) v *= dz;
    return v;
}

// ------------------------------------------------------------ far field
// T_n(R) by eq. 3.4 with T_0 = 1/|R|:
//   T_n = -[ (2s-1)/s sum_i R_i T_{n-e_i} + (s-1)/s sum_i T_{n-2e_i} ] / |R|^2.
template <int K, int N>
__device__ __forceinline__ void t_step(double (&T)[N], double Rx, double Ry, double Rz, double ir2) {
    constexpr TEnt e = TT1.e[K];
    double f = 0.0, g = 0.0;
    if constexpr (e.x1 >= 0) f = Rx * T[e.x1];
    if constexpr (e.y1 >= 0) f = fma(Ry, T[e.y1], f);
    if constexpr (e.z1 >= 0) f = fma(Rz, T[e.z1], f);
    if constexpr (e.x2 >= 0) g = T[e.x2];
    if constexpr (e.y2 >= 0) g += T[e.y2];
    if constexpr (e.z2 >= 0) g += T[e.z2];
    constexpr double A = (2.0 * e.s - 1.0) / e.s;
    constexpr double B = (e.s - 1.0) / e.s;
    if constexpr (e.s >= 2) T[K] = -fma(A, f, B * g) * ir2;
    else T[K] = -(A * f) * ir2;
}

// Moment rows are read through pointers qualified with their address space:
// global (HBM) rows then compile to global loads and LDS rows to LDS loads, each
// waited for by its own counter, so several of a row's loads are in flight at
// once.  Through a generic pointer they become flat loads, each waited for in
// full before the next is issued.
using GRow = const __attribute__((address_space(1))) double*;
using LRow = const __attribute__((address_space(3))) double*;
__device__ __forceinline__ GRow grow(const double* p) { return (GRow)p; }
__device__ __forceinline__ LRow lrow(const double* p) { return (LRow)p; }

// An FP64 add to HBM through a global-qualified pointer: the compiler then knows
// it cannot write LDS, so LDS loads stay free to move across it.
using GDbl = __attribute__((address_space(1))) double*;
__device__ __forceinline__ void gatomic_add(double* p, double v) { __builtin_amdgcn_global_atomic_fadd_f64((GDbl)p, v); }

// The same for single records of the tree in HBM: cell geometry, cell header,
// a source, a slot's source index, a tracking entry.
using GInt = const __attribute__((address_space(1))) int*;
__device__ __forceinline__ double4 gload(const double4* p) {
    const GRow q = (GRow)(const double*)p;
    return make_double4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ int4 gload(const int4* p) {
    const GInt q = (GInt)(const int*)p;
    return make_int4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ int2 gload(const int2* p) {
    const GInt q = (GInt)(const int*)p;
    return make_int2(q[0], q[1]);
}
__device__ __forceinline__ int gload(const int* p) { return *(GInt)p; }

// sum_n T_n M^n, each T_n folded into the sum as soon as it exists
template <int K, class MP>
__device__ __forceinline__ void far_rec(double (&T)[NTERM], double Rx, double Ry, double Rz,
                                        double ir2, MP __restrict__ Mc, double& acc) {
    if constexpr (K < NTERM) {
        if constexpr (K > 0) t_step<K>(T, Rx, Ry, Rz, ir2);
        acc = fma(T[K], Mc[K], acc);
        far_rec<K + 1>(T, Rx, Ry, Rz, ir2, Mc, acc);
    }
}

template <class MP>
__device__ __forceinline__ double far_eval(double Rx, double Ry, double Rz, MP Mc) {
    const double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    double T[NTERM];
    T[0] = rsqrt_nr(r2);
    const double ir2 = T[0] * T[0];
    double acc = 0.0;
    far_rec<0>(T, Rx, Ry, Rz, ir2, Mc, acc);
    return acc;
}

// The same in single precision from the single-precision moments: T_n by eq. 3.4 in
// FP32 and sum_n T_n M^n accumulated in FP32 per cell (the caller adds the cell's value
// to an FP64 sum).
template <int K>
__device__ __forceinline__ void t_step_f(float (&T)[NTERM], float Rx, float Ry, float Rz, float ir2) {
    constexpr TEnt e = TT.e[K];
    float f = 0.0f, g = 0.0f;
    if constexpr (e.x1 >= 0) f = Rx * T[e.x1];
    if constexpr (e.y1 >= 0) f = fmaf(Ry, T[e.y1], f);
    if constexpr (e.z1 >= 0) f = fmaf(Rz, T[e.z1], f);
    if constexpr (e.x2 >= 0) g = T[e.x2];
    if constexpr (e.y2 >= 0) g += T[e.y2];
    if constexpr (e.z2 >= 0) g += T[e.z2];
    constexpr float A = (float)((2.0 * e.s - 1.0) / e.s);
    constexpr float B = (float)((e.s - 1.0) / e.s);
    if constexpr (e.s >= 2) T[K] = -fmaf(A, f, B * g) * ir2;
    else T[K] = -(A * f) * ir2;
}

template <int K>
__device__ __forceinline__ void far_rec_f(float (&T)[NTERM], float Rx, float Ry, float Rz, float ir2,
                                          const __attribute__((address_space(1))) float* __restrict__ Mc, float& acc) {
    if constexpr (K < NTERM) {
        if constexpr (K > 0) t_step_f<K>(T, Rx, Ry, Rz, ir2);
        acc = fmaf(T[K], Mc[K], acc);
        far_rec_f<K + 1>(T, Rx, Ry, Rz, ir2, Mc, acc);
    }
}

__device__ __forceinline__ double far_eval_f(double Rx, double Ry, double Rz, const float* M32row) {
    const float rx = (float)Rx, ry = (float)Ry, rz = (float)Rz;
    const float r2 = rx * rx + ry * ry + rz * rz;
    float T[NTERM];
    T[0] = __builtin_amdgcn_rsqf(r2);
    T[0] = T[0] * fmaf(-0.5f * r2 * T[0], T[0], 1.5f);  // one Newton step
    const float ir2 = T[0] * T[0];
    float acc = 0.0f;
    far_rec_f<0>(T, rx, ry, rz, ir2, (const __attribute__((address_space(1))) float*)M32row, acc);
    return (double)acc;
}

// Far value of cell c at relative position R: FP32 from M32 when the replica keeps it.
__device__ __forceinline__ double far_value(const Rep& R, int c, double Rx, double Ry, double Rz) {
    if (R.M32) return far_eval_f(Rx, Ry, Rz, R.M32 + (size_t)c * MSTR);
    return far_eval(Rx, Ry, Rz, grow(R.M + (size_t)c * MSTR));
}

// Polynomial sum_n C_n d^n and its gradient sum_n C_n n_k d^{n - e_k} for
// stored coefficients C; the monomials d^n are built by the graded
// recurrence, each from one of order |n| - 1.
template <int K>
__device__ __forceinline__ void poly_rec(double (&D)[NTERM], double dx, double dy, double dz,
                                         const double* __restrict__ Cc, double& v, double& gx, double& gy,
                                         double& gz) {
    if constexpr (K < NTERM) {
        constexpr TEnt e = TT.e[K];
        const double c = Cc[K];
        if constexpr (K == 0) D[0] = 1.0;
        else if constexpr (e.n1 >= 1) D[K] = D[e.x1] * dx;
        else if constexpr (e.n2 >= 1) D[K] = D[e.y1] * dy;
        else D[K] = D[e.z1] * dz;
        v = fma(c, D[K], v);
        if constexpr (e.x1 >= 0) gx = fma((double)e.n1 * c, D[e.x1], gx);
        if constexpr (e.y1 >= 0) gy = fma((double)e.n2 * c, D[e.y1], gy);
        if constexpr (e.z1 >= 0) gz = fma((double)e.n3 * c, D[e.z1], gz);
        poly_rec<K + 1>(D, dx, dy, dz, Cc, v, gx, gy, gz);
    }
}

// ------------------------------------------------------------ traversal state
constexpr uint32_t kCellMask = 0xFFFFFFu;
constexpr uint32_t kFlagIon = 1u << 28, kFlagImg = 1u << 29, kFlagDirect = 1u << 30;

__device__ __forceinline__ uint32_t pack(int cell, int t, uint32_t flags) {
    return (uint32_t)cell | ((uint32_t)t << 24) | flags;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Frontier region of this workgroup in HBM (null if none): a level whose frontier
// outgrows its LDS capacity continues there, and so do the levels after it.
__device__ __forceinline__ uint32_t* spill_region(const Rep& R) {
    return (R.spill && (int)blockIdx.x < R.spill_regions) ? R.spill + (size_t)blockIdx.x * (size_t)R.spill_words
                                                          : nullptr;
}

template <int NTG, int BLOCK>
struct Trav {
    static constexpr int FCAP = 4096;
    static constexpr int FARCAP = 1024 + BLOCK;
    static constexpr int NEARCAP = 512 + BLOCK;
    static constexpr int OVLCAP = 256;
    static constexpr int NW = BLOCK / 64;
    uint32_t front[2][FCAP];
    uint32_t farl[FARCAP];
    uint32_t nearl[NEARCAP];
    int near_base[NEARCAP];
    int near_pre[NEARCAP + 1];       // slot counts, then their exclusive prefix
    uint32_t flagl[2 * NTG];
    double Mx[2 * NTG][MSTR];
    double tx[NTG], ty[NTG], tz[NTG];
    int ex_i[NTG], ex_k[NTG];
    uint64_t kx_i[NTG], kx_k[NTG];
    double4 es_i[NTG], es_k[NTG];
    uint32_t ovl[OVLCAP];
    int n_ovl, ovl_t, ovl_ex;
    int near_tot;                    // slot total of the near leaves, from a one-wave scan
    int err, overlap, coincide;
    uint64_t wcnt[2][NW];            // per-wave packed list counts, double buffered
    uint64_t wsum[NW + 1];
    double red[NW][NTG];
    double res[NTG];
    uint32_t mi[NTERM];              // multi-index of each term, packed (mi_code)
};

template <int NTG, int BLOCK>
__device__ __forceinline__ void fill_mi(Trav<NTG, BLOCK>& S) {
    for (int k = threadIdx.x; k < NTERM; k += BLOCK) S.mi[k] = mi_code(k);
}

template <int NTG>
__device__ __forceinline__ void add_to(double (&acc)[NTG], int t, double v) {
#pragma unroll
    for (int k = 0; k < NTG; ++k)
        if (k == t) acc[k] += v;
}

// Far cells, then the cells holding an excluded source, whose corrected
// moments sit in LDS.
template <int NTG, int BLOCK>
__device__ __forceinline__ void far_pass(const Rep& R, Trav<NTG, BLOCK>& S, int far_n, int nflag,
                                         double (&acc)[NTG]) {
    for (int j = threadIdx.x; j < far_n; j += BLOCK) {
        const uint32_t e = S.farl[j];
        const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const double4 g = R.cgeo[c];
        add_to<NTG>(acc, t, far_value(R, c, g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t]));
    }
    for (int j = threadIdx.x; j < nflag; j += BLOCK) {
        const uint32_t e = S.flagl[j];
        const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const double4 g = R.cgeo[c];
        add_to<NTG>(acc, t, far_eval(g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t], lrow(S.Mx[j])));
    }
}

// Exclusive scan of the near leaves' slot counts (in place in near_pre).  Up to
// 64 leaves (the usual case) the first wave scans them by shuffles and one
// barrier publishes the result; beyond that, block scans of BLOCK at a time.
template <int NTG, int BLOCK>
__device__ int near_scan(Trav<NTG, BLOCK>& S, int near_n) {
    if (near_n <= 64) {  // uniform
        if (threadIdx.x < 64) {
            const int j = threadIdx.x;
            const int v = j < near_n ? S.near_pre[j] : 0;
            int x = v;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(x, off, 64);
                if (j >= off) x += y;
            }
            if (j < near_n) S.near_pre[j] = x - v;
            if (j == 63) S.near_tot = x;
        }
        __syncthreads();
        return S.near_tot;
    }
    int carry = 0;
    for (int base = 0; base < near_n; base += BLOCK) {
        const int j = base + threadIdx.x;
        const int v = j < near_n ? S.near_pre[j] : 0;
        uint64_t tot;
        const uint64_t ex = block_exscan<BLOCK>((uint64_t)v, S.wsum, tot);
        if (j < near_n) S.near_pre[j] = carry + (int)ex;
        carry += (int)tot;
        __syncthreads();
    }
    return carry;
}

// Near leaves: direct sum over each leaf's index array in slot order.  For
// the overlap target, every ion other than the mover within tau is an overlap.
template <int NTG, int BLOCK>
__device__ __forceinline__ void near_pass(const Rep& R, Trav<NTG, BLOCK>& S, int near_n, int total,
                                          double (&acc)[NTG]) {
    const int n_ion = R.n;
    for (int f = threadIdx.x; f < total; f += BLOCK) {
        int lo = 0, hi = near_n - 1;  // last j with near_pre[j] <= f
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.near_pre[mid] <= f) lo = mid; else hi = mid - 1;
        }
        const uint32_t e = S.nearl[lo];
        const int t = (int)((e >> 24) & 15u);
        const int slot = S.near_base[lo] + (f - S.near_pre[lo]);
        const double4 s = R.pool4[slot];
        const bool check_ovl = (t == S.ovl_t);
        int sid = -1;
        if ((e & (kFlagIon | kFlagImg)) || check_ovl) {
            sid = R.pidx[slot];
            if (((e & kFlagIon) && sid == S.ex_i[t]) || ((e & kFlagImg) && sid == S.ex_k[t])) continue;
        }
        const double dx = S.tx[t] - s.x, dy = S.ty[t] - s.y, dz = S.tz[t] - s.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (check_ovl && sid < n_ion && sid != S.ovl_ex && d2 <= R.tau2) S.overlap = 1;
        if (d2 == 0.0) { S.coincide = 1; continue; }
        add_to<NTG>(acc, t, s.w * rsqrt_nr(d2));
    }
}

// squared distance from a point to the closed cube of centre g and half side g.w
__device__ __forceinline__ double box_dist2(double4 g, double x, double y, double z) {
    double ax = fabs(x - g.x) - g.w, ay = fabs(y - g.y) - g.w, az = fabs(z - g.z) - g.w;
    ax = ax > 0.0 ? ax : 0.0; ay = ay > 0.0 ? ay : 0.0; az = az > 0.0 ? az : 0.0;
    return ax * ax + ay * ay + az * az;
}

// Hard-core check below cells the traversal took as far: descend every cell
// whose cube comes within tau (plus a rounding margin) of the target.
template <int NTG, int BLOCK>
__device__ void overlap_below_far(const Rep& R, Trav<NTG, BLOCK>& S, int* cnt2) {
    using TS = Trav<NTG, BLOCK>;
    const int t = S.ovl_t;
    const double x = S.tx[t], y = S.ty[t], z = S.tz[t];
    const double reach2 = R.reach2;
    // n_ovl counts every insert attempt; entries past OVLCAP were never stored
    int cur = 0, fs = S.n_ovl < TS::OVLCAP ? S.n_ovl : TS::OVLCAP;
    for (int j = threadIdx.x; j < fs; j += BLOCK) S.front[0][j] = S.ovl[j];
    while (fs > 0) {
        if (threadIdx.x == 0) cnt2[cur ^ 1] = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < fs; j += BLOCK) {
            const int c = (int)S.front[cur][j];
            if (c < 0 || c >= R.ncell) { S.err = kErrOvlLeaf; continue; }
            const int4 m = R.cm[c];
            if (m.y >= 0 && m.y + 8 > R.ncell) { S.err = kErrChildLink; continue; }
            if (m.y < 0) {
                if (m.x < 0 || m.z < 0 || m.z + m.x > R.pool) { S.err = kErrOvlLeaf; continue; }
                for (int k = 0; k < m.x; ++k) {
                    const int sid = R.pidx[m.z + k];
                    if (sid >= R.n || sid == S.ovl_ex) continue;
                    const double4 s = R.pool4[m.z + k];
                    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
                    if (dx * dx + dy * dy + dz * dz <= R.tau2) S.overlap = 1;
                }
            } else {
                for (int d = 0; d < 8; ++d) {
                    const int ch = m.y + d;
                    if (R.cm[ch].x == 0) continue;
                    if (box_dist2(R.cgeo[ch], x, y, z) <= reach2) {
                        const int slot = atomicAdd(&cnt2[cur ^ 1], 1);
                        if (slot < TS::FCAP) S.front[cur ^ 1][slot] = (uint32_t)ch;
                        else S.err = kErrStack;
                    }
                }
            }
        }
        __syncthreads();
        fs = cnt2[cur ^ 1];
        if (fs > TS::FCAP) fs = TS::FCAP;
        cur ^= 1;
        __syncthreads();
    }
}

// Breadth-first MAC traversal (Sec. 3.2) from the entries already in
// front[0].  Each chunk of BLOCK entries is classified lane by lane; wave
// ballots and one barrier hand out list slots in a fixed order, so every sum
// below is taken in the same order on every run.  On return S.res[t] holds
// the potential at target t from every source except the target's excluded
// ones; S.err reports an overflowed list or a failed index check;
// S.overlap / S.coincide report hard-core hits at the overlap target.
// Returns the number of levels processed (hook is called once per level,
// by every thread, right after the level's first loads are issued).
template <int NTG, int BLOCK, class Hook>
__device__ int traverse(const Rep& R, Trav<NTG, BLOCK>& S, int nroot, int* cnt2, Hook&& hook) {
    using TS = Trav<NTG, BLOCK>;
    constexpr int NW = TS::NW;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    double acc[NTG];
#pragma unroll
    for (int k = 0; k < NTG; ++k) acc[k] = 0.0;
    int cur = 0, fs = nroot, far_n = 0, near_n = 0, nflag = 0, buf = 0;
    bool failed = false, frontier_full = false;
    // the frontier: front[] in LDS up to lcap entries, then the workgroup's HBM region (two halves
    // of gcap entries); rg / wg: the level read / the level written is in HBM (uniform)
    uint32_t* const gfr = spill_region(R);
    const int gcap = gfr ? (int)(R.spill_words / 2 < 0x7FFFFFFF ? R.spill_words / 2 : 0x7FFFFFFF) : 0;
    const int lcap = R.fcap < TS::FCAP ? R.fcap : TS::FCAP;
    bool rg = false, wg = false;
    int level = 0;
    for (; fs > 0 && !failed; ++level) {
        int next_n = 0;
        for (int base = 0; base < fs; base += BLOCK) {
            if (far_n > TS::FARCAP - BLOCK) {
                __syncthreads();
                far_pass<NTG, BLOCK>(R, S, far_n, 0, acc);
                far_n = 0;
                __syncthreads();
            }
            if (near_n > TS::NEARCAP - BLOCK) {
                __syncthreads();
                const int total = near_scan<NTG, BLOCK>(S, near_n);
                near_pass<NTG, BLOCK>(R, S, near_n, total, acc);
                near_n = 0;
                __syncthreads();
            }
            const int j = base + tid;
            const bool valid = j < fs;
            const uint32_t e = valid ? (rg ? gfr[(size_t)cur * gcap + j] : S.front[cur][j]) : 0u;
            const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
            const int fi = (e & kFlagIon) ? 1 : 0, fk = (e & kFlagImg) ? 1 : 0;
            int kind = 0;
            int4 m = make_int4(0, -1, 0, 0);
            double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
            if (valid && c < R.ncell) { m = R.cm[c]; g = R.cgeo[c]; }
            // once per level, in the shadow of the loads just issued
            if (base == 0) hook(level);
            uint32_t cdir = e & kFlagDirect;
            if (valid && c >= R.ncell) {
                S.err = kErrFrontCell;
            } else if (valid) {
                const int np = m.x - fi - fk;
                if (m.y >= 0 && m.y + 8 > R.ncell) {
                    S.err = kErrChildLink;
                } else if (np > 0) {
                    if (cdir) {
                        kind = m.y >= 0 ? 3 : 2;
                    } else {
                        const double dx = g.x - S.tx[t], dy = g.y - S.ty[t], dz = g.z - S.tz[t];
                        const double d2 = dx * dx + dy * dy + dz * dz;
                        const bool mac = 3.0 * (g.w * g.w) <= R.theta2 * d2;
                        if (mac && np >= R.n0) {
                            kind = (fi | fk) ? 4 : 1;
                            if (t == S.ovl_t) {
                                if (box_dist2(g, S.tx[t], S.ty[t], S.tz[t]) <= R.reach2) {
                                    const int slot = atomicAdd(&S.n_ovl, 1);
                                    if (slot < TS::OVLCAP) S.ovl[slot] = (uint32_t)c; else S.err = kErrStack;
                                }
                            }
                        } else if (np > R.n0 && m.y >= 0) {
                            kind = 3;
                        } else if (m.y < 0) {
                            kind = 2;
                        } else {
                            kind = 3;
                            cdir = kFlagDirect;  // N_A <= N_0: sum every source below directly
                        }
                    }
                }
            }
            const uint64_t lt = lanemask_lt();
            const uint64_t bf = __ballot(kind == 1), bn = __ballot(kind == 2);
            const uint64_t bs = __ballot(kind == 3), bg = __ballot(kind == 4);
            if (lane == 0)
                S.wcnt[buf][w] = (uint64_t)__popcll(bf) | ((uint64_t)__popcll(bn) << 16) |
                                 ((uint64_t)__popcll(bs) << 32) | ((uint64_t)__popcll(bg) << 48);
            __syncthreads();
            uint64_t before = 0, tot = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint64_t v = S.wcnt[buf][ww];
                before += ww < w ? v : 0ull;
                tot += v;
            }
            buf ^= 1;
            const int tf = (int)(tot & 0xffff), tn = (int)((tot >> 16) & 0xffff);
            const int ts = (int)((tot >> 32) & 0xffff), tg = (int)(tot >> 48);
            if (nflag + tg > 2 * NTG) {  // uniform
                failed = true;
                break;
            }
            if (next_n + 8 * ts > (wg ? gcap : lcap)) {  // uniform
                if (wg || next_n + 8 * ts > gcap) {
                    failed = frontier_full = true;
                    break;
                }
                // the next level moves to HBM: what this level wrote so far first
                for (int k = tid; k < next_n; k += BLOCK) gfr[(size_t)(cur ^ 1) * gcap + k] = S.front[cur ^ 1][k];
                wg = true;
            }
            if (kind == 1) {
                S.farl[far_n + (int)(before & 0xffff) + __popcll(bf & lt)] = e;
            } else if (kind == 2) {
                const int o = near_n + (int)((before >> 16) & 0xffff) + __popcll(bn & lt);
                S.nearl[o] = e;
                S.near_base[o] = m.z;
                S.near_pre[o] = m.x;
                if (m.x < 0 || m.z < 0 || m.z + m.x > R.pool) { S.near_pre[o] = 0; S.err = kErrNearSlots; }
            } else if (kind == 4) {
                S.flagl[nflag + (int)(before >> 48) + __popcll(bg & lt)] = e;
            } else if (kind == 3) {
                const int o = next_n + 8 * ((int)((before >> 32) & 0xffff) + __popcll(bs & lt));
                const int dig_i = fi ? key_digit(S.kx_i[t], level + 1) : -1;
                const int dig_k = fk ? key_digit(S.kx_k[t], level + 1) : -1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const uint32_t fl = (d == dig_i ? kFlagIon : 0u) | (d == dig_k ? kFlagImg : 0u) | cdir;
                    if (wg) gfr[(size_t)(cur ^ 1) * gcap + o + d] = pack(m.y + d, t, fl);
                    else S.front[cur ^ 1][o + d] = pack(m.y + d, t, fl);
                }
            }
            far_n += tf; near_n += tn; nflag += tg; next_n += 8 * ts;
        }
        __syncthreads();  // the next level reads what this one wrote
        cur ^= 1;
        fs = next_n;
        rg = wg;
    }
    if (failed) {
        if (tid == 0) S.err = frontier_full ? kErrFrontier : kErrStack;
        __syncthreads();
        return level;
    }
    // corrected moments of the far cells that hold an excluded source
    for (int it = tid; it < nflag * NTERM; it += BLOCK) {
        const int f = it / NTERM, k = it % NTERM;
        const uint32_t e = S.flagl[f];
        const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
        if (c >= R.ncell) { S.err = kErrFlagCell; S.Mx[f][k] = 0.0; continue; }
        const double4 g = R.cgeo[c];
        double mk = R.M[(size_t)c * MSTR + k];
        if (e & kFlagIon) { const double4 s = S.es_i[t]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        if (e & kFlagImg) { const double4 s = S.es_k[t]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        S.Mx[f][k] = mk;
    }
    const int total = near_scan<NTG, BLOCK>(S, near_n);  // its barriers also publish Mx
    far_pass<NTG, BLOCK>(R, S, far_n, nflag, acc);
    near_pass<NTG, BLOCK>(R, S, near_n, total, acc);
    __syncthreads();
    if (S.ovl_t >= 0 && S.n_ovl > 0 && S.err == 0) overlap_below_far<NTG, BLOCK>(R, S, cnt2);
#pragma unroll
    for (int k = 0; k < NTG; ++k) {
        const double sum = wave_sum(acc[k]);
        if (lane == 0) S.red[w][k] = sum;
    }
    __syncthreads();
    if (tid < NTG) {
        double sum = 0.0;
        for (int ww = 0; ww < NW; ++ww) sum += S.red[ww][tid];
        S.res[tid] = sum;
    }
    __syncthreads();
    return level;
}

// ------------------------------------------------------------ the move traversal
// The two targets of a move (the mover's old and new position) exclude the
// same two sources, so they share every frontier entry: a cell with a 2-bit
// mask of the targets for which it is still open (bits 24-25), a 2-bit mask of
// the targets summing every source below it directly by the N_0 rule (bits
// 26-27) and the two exclusion flags.  Each target takes exactly the decisions
// of its own traversal.  Far cells are evaluated by lane pairs (lane 2j the
// old position, 2j+1 the new one) reading the same moment row; near sources by
// lanes that load a source once and evaluate both targets against it.
constexpr int kMaskSh = 24, kDirSh = 26;

template <int BLOCK>
__device__ __forceinline__ void far_pass_mc(const Rep& R, Trav<2, BLOCK>& S, int far_n, int nflag,
                                            double (&acc)[2]) {
    static_assert(BLOCK % 2 == 0, "lane pairs");
    const int t = (int)(threadIdx.x & 1);
    for (int j2 = threadIdx.x; j2 < 2 * far_n; j2 += BLOCK) {
        const uint32_t e = S.farl[j2 >> 1];
        if (!((e >> (kMaskSh + t)) & 1u)) continue;
        const int c = (int)(e & kCellMask);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const double4 g = R.cgeo[c];
        add_to<2>(acc, t, far_value(R, c, g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t]));
    }
    // the cells holding an excluded source, with their corrected moments in LDS
    for (int j2 = threadIdx.x; j2 < 2 * nflag; j2 += BLOCK) {
        const uint32_t e = S.flagl[j2 >> 1];
        if (!((e >> (kMaskSh + t)) & 1u)) continue;
        const int c = (int)(e & kCellMask);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const double4 g = R.cgeo[c];
        add_to<2>(acc, t, far_eval(g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t], lrow(S.Mx[j2 >> 1])));
    }
}

// Near leaves of both targets.  For the new position (the overlap target),
// every ion other than the mover within tau is an overlap.
template <int BLOCK>
__device__ __forceinline__ void near_pass_mc(const Rep& R, Trav<2, BLOCK>& S, int near_n, int total,
                                             double (&acc)[2]) {
    const int n_ion = R.n;
    for (int f = threadIdx.x; f < total; f += BLOCK) {
        int lo = 0, hi = near_n - 1;  // last j with near_pre[j] <= f
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.near_pre[mid] <= f) lo = mid; else hi = mid - 1;
        }
        const uint32_t e = S.nearl[lo];
        const uint32_t mask = (e >> kMaskSh) & 3u;
        const int slot = S.near_base[lo] + (f - S.near_pre[lo]);
        const double4 s = gload(R.pool4 + slot);
        int sid = -1;
        if ((e & (kFlagIon | kFlagImg)) || (mask & 2u)) {
            sid = gload(R.pidx + slot);
            if (((e & kFlagIon) && sid == S.ex_i[0]) || ((e & kFlagImg) && sid == S.ex_k[0])) continue;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (!((mask >> t) & 1u)) continue;
            const double dx = S.tx[t] - s.x, dy = S.ty[t] - s.y, dz = S.tz[t] - s.z;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (t == 1 && sid < n_ion && sid != S.ovl_ex && d2 <= R.tau2) S.overlap = 1;
            if (d2 == 0.0) { S.coincide = 1; continue; }
            add_to<2>(acc, t, s.w * rsqrt_nr(d2));
        }
    }
}

// Breadth-first MAC traversal (Sec. 3.2) of the two targets of a move from
// the fs0 entries of level level0 in front[0]; otherwise as traverse():
// deterministic lists, hook once per level, res[0..1] the potentials (the
// same in every thread), S.err / S.overlap / S.coincide as there.
template <int BLOCK, class Hook>
__device__ int traverse_mc(const Rep& R, Trav<2, BLOCK>& S, int* cnt2, Hook&& hook, int fs0, int level0,
                           double (&res)[2]) {
    using TS = Trav<2, BLOCK>;
    res[0] = res[1] = 0.0;
    constexpr int NW = TS::NW;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    double acc[2] = {0.0, 0.0};
    int cur = 0, fs = fs0, far_n = 0, near_n = 0, nflag = 0, buf = 0;
    bool failed = false, frontier_full = false;
    // the frontier: LDS up to lcap entries, then HBM (see traverse)
    uint32_t* const gfr = spill_region(R);
    const int gcap = gfr ? (int)(R.spill_words / 2 < 0x7FFFFFFF ? R.spill_words / 2 : 0x7FFFFFFF) : 0;
    const int lcap = R.fcap < TS::FCAP ? R.fcap : TS::FCAP;
    bool rg = false, wg = false;
    int level = level0;
    for (; fs > 0 && !failed; ++level) {
        int next_n = 0;
        for (int base = 0; base < fs; base += BLOCK) {
            if (far_n > TS::FARCAP - BLOCK) {
                __syncthreads();
                far_pass_mc<BLOCK>(R, S, far_n, 0, acc);
                far_n = 0;
                __syncthreads();
            }
            if (near_n > TS::NEARCAP - BLOCK) {
                __syncthreads();
                const int total = near_scan<2, BLOCK>(S, near_n);
                near_pass_mc<BLOCK>(R, S, near_n, total, acc);
                near_n = 0;
                __syncthreads();
            }
            const int j = base + tid;
            const bool valid = j < fs;
            const uint32_t e = valid ? (rg ? gfr[(size_t)cur * gcap + j] : S.front[cur][j]) : 0u;
            const int c = (int)(e & kCellMask);
            const int fi = (e & kFlagIon) ? 1 : 0, fk = (e & kFlagImg) ? 1 : 0;
            const uint32_t open = (e >> kMaskSh) & 3u, dir = (e >> kDirSh) & 3u;
            int4 m = make_int4(0, -1, 0, 0);
            double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
            if (valid && c < R.ncell) { m = gload(R.cm + c); g = gload(R.cgeo + c); }
            // once per level, in the shadow of the loads just issued
            if (base == 0) hook(level);
            uint32_t farb = 0, nearb = 0, copen = 0, cdir = 0;
            if (valid && c >= R.ncell) {
                S.err = kErrFrontCell;
            } else if (valid) {
                const int np = m.x - fi - fk;
                if (m.y >= 0 && m.y + 8 > R.ncell) {
                    S.err = kErrChildLink;
                } else if (np > 0) {
                    // both targets' tests side by side, then the decisions as bit masks
                    const double dx0 = g.x - S.tx[0], dy0 = g.y - S.ty[0], dz0 = g.z - S.tz[0];
                    const double dx1 = g.x - S.tx[1], dy1 = g.y - S.ty[1], dz1 = g.z - S.tz[1];
                    const double d20 = dx0 * dx0 + dy0 * dy0 + dz0 * dz0;
                    const double d21 = dx1 * dx1 + dy1 * dy1 + dz1 * dz1;
                    const double h2 = 3.0 * (g.w * g.w);
                    const uint32_t mac = (h2 <= R.theta2 * d20 ? 1u : 0u) | (h2 <= R.theta2 * d21 ? 2u : 0u);
                    const bool internal = m.y >= 0;
                    const uint32_t live = open & ~dir;
                    farb = live & mac & (np >= R.n0 ? 3u : 0u);
                    const uint32_t rest = live & ~farb;
                    copen = rest & ((np > R.n0 && internal) ? 3u : 0u);
                    nearb = (rest & ~copen & (internal ? 0u : 3u)) | (dir & (internal ? 0u : 3u));
                    cdir = (rest & ~copen & (internal ? 3u : 0u)) | (dir & (internal ? 3u : 0u));
                    if ((farb & 2u) && S.ovl_t == 1 && box_dist2(g, S.tx[1], S.ty[1], S.tz[1]) <= R.reach2) {
                        const int slot = atomicAdd(&S.n_ovl, 1);
                        if (slot < TS::OVLCAP) S.ovl[slot] = (uint32_t)c; else S.err = kErrStack;
                    }
                }
            }
            const bool flagged = (fi | fk) != 0;
            const bool kf = farb && !flagged, kg = farb && flagged, kn = nearb != 0, ks = (copen | cdir) != 0;
            const uint64_t lt = lanemask_lt();
            const uint64_t bf = __ballot(kf), bn = __ballot(kn), bs = __ballot(ks), bg = __ballot(kg);
            if (lane == 0)
                S.wcnt[buf][w] = (uint64_t)__popcll(bf) | ((uint64_t)__popcll(bn) << 16) |
                                 ((uint64_t)__popcll(bs) << 32) | ((uint64_t)__popcll(bg) << 48);
            __syncthreads();
            uint64_t before = 0, tot = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint64_t v = S.wcnt[buf][ww];
                before += ww < w ? v : 0ull;
                tot += v;
            }
            buf ^= 1;
            const int tf = (int)(tot & 0xffff), tn = (int)((tot >> 16) & 0xffff);
            const int ts = (int)((tot >> 32) & 0xffff), tg = (int)(tot >> 48);
            if (nflag + tg > 4) {  // uniform
                failed = true;
                break;
            }
            if (next_n + 8 * ts > (wg ? gcap : lcap)) {  // uniform
                if (wg || next_n + 8 * ts > gcap) {
                    failed = frontier_full = true;
                    break;
                }
                for (int k = tid; k < next_n; k += BLOCK) gfr[(size_t)(cur ^ 1) * gcap + k] = S.front[cur ^ 1][k];
                wg = true;
            }
            const uint32_t flags = e & (kFlagIon | kFlagImg);
            if (kf) S.farl[far_n + (int)(before & 0xffff) + __popcll(bf & lt)] = (uint32_t)c | (farb << kMaskSh);
            if (kg) S.flagl[nflag + (int)(before >> 48) + __popcll(bg & lt)] = (uint32_t)c | (farb << kMaskSh) | flags;
            if (kn) {
                const int o = near_n + (int)((before >> 16) & 0xffff) + __popcll(bn & lt);
                S.nearl[o] = (uint32_t)c | (nearb << kMaskSh) | flags;
                S.near_base[o] = m.z;
                S.near_pre[o] = m.x;
                if (m.x < 0 || m.z < 0 || m.z + m.x > R.pool) { S.near_pre[o] = 0; S.err = kErrNearSlots; }
            }
            if (ks) {
                const int o = next_n + 8 * ((int)((before >> 32) & 0xffff) + __popcll(bs & lt));
                const int dig_i = fi ? key_digit(S.kx_i[0], level + 1) : -1;
                const int dig_k = fk ? key_digit(S.kx_k[0], level + 1) : -1;
                const uint32_t masks = (copen << kMaskSh) | (cdir << kDirSh);
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const uint32_t fl = (d == dig_i ? kFlagIon : 0u) | (d == dig_k ? kFlagImg : 0u);
                    if (wg) gfr[(size_t)(cur ^ 1) * gcap + o + d] = (uint32_t)(m.y + d) | masks | fl;
                    else S.front[cur ^ 1][o + d] = (uint32_t)(m.y + d) | masks | fl;
                }
            }
            far_n += tf; near_n += tn; nflag += tg; next_n += 8 * ts;
        }
        __syncthreads();  // the next level reads what this one wrote
        cur ^= 1;
        fs = next_n;
        rg = wg;
    }
    if (failed) {
        if (tid == 0) S.err = frontier_full ? kErrFrontier : kErrStack;
        __syncthreads();
        return level;
    }
    // corrected moments of the far cells that hold an excluded source
    for (int it = tid; it < nflag * NTERM; it += BLOCK) {
        const int f = it / NTERM, k = it % NTERM;
        const uint32_t e = S.flagl[f];
        const int c = (int)(e & kCellMask);
        if (c >= R.ncell) { S.err = kErrFlagCell; S.Mx[f][k] = 0.0; continue; }
        const double4 g = R.cgeo[c];
        double mk = R.M[(size_t)c * MSTR + k];
        if (e & kFlagIon) { const double4 s = S.es_i[0]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        if (e & kFlagImg) { const double4 s = S.es_k[0]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        S.Mx[f][k] = mk;
    }
    const int total = near_scan<2, BLOCK>(S, near_n);  // its barriers also publish Mx
    far_pass_mc<BLOCK>(R, S, far_n, nflag, acc);
    near_pass_mc<BLOCK>(R, S, near_n, total, acc);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double sum = wave_sum(acc[k]);
        if (lane == 0) S.red[w][k] = sum;
    }
    __syncthreads();
    if (S.ovl_t >= 0 && S.n_ovl > 0 && S.err == 0) overlap_below_far<2, BLOCK>(R, S, cnt2);
    // every thread sums the wave sums itself, in the same order
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double sum = 0.0;
        for (int ww = 0; ww < NW; ++ww) sum += S.red[ww][k];
        res[k] = sum;
    }
    return level;
}

// sum_{s <= p} P_s(cos psi) |d|^s / |R|^(s+1), psi the angle between d and -R: the
// expansion of eq. 3.3 of one unit point source at c + d seen from c - R, order by
// order equal to sum_{|n| <= p} T_n(R) d^n.  With A_s = P_s(cos psi) |d|^s |R|^s,
// (s + 1) A_{s+1} = (2s + 1) (-d.R) A_s - s |d|^2 |R|^2 A_{s-1}.
__device__ __forceinline__ double point_expansion(double Rx, double Ry, double Rz, double dx, double dy, double dz) {
    const double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    const double ir = rsqrt_nr(r2);
    const double irr = ir * ir;
    const double c1 = -(dx * Rx + dy * Ry + dz * Rz);
    const double c2 = (dx * dx + dy * dy + dz * dz) * r2;
    double a0 = 1.0, a1 = c1;
    double sc = ir;               // |R|^-(2s+1)
    double v = a0 * sc;
    if (P >= 1) { sc *= irr; v = fma(a1, sc, v); }
#pragma unroll
    for (int s = 1; s < P; ++s) {
        const double a2 = ((2.0 * s + 1.0) * c1 * a1 - (double)s * c2 * a0) / (s + 1.0);
        a0 = a1; a1 = a2;
        sc *= irr;
        v = fma(a1, sc, v);
    }
    return v;
}

// What a unit source at sc adds to the potential at (x, y, z) through the tree when
// the traversal keeps it as an ordinary source (N_0 = 0): walk its root path from the
// top; the first cell passing the MAC takes it through its expansion, otherwise its
// leaf takes it directly.  bad is set (and 0 returned) where a link is broken.
__device__ __forceinline__ double walk_value(const Rep& R, double4 sc, double x, double y, double z, int& bad) {
    const uint64_t key = morton_key(R, sc.x, sc.y, sc.z);
    int c = 0;
    for (int level = 0; level < kMaxLevels; ++level) {
        if (c < 0 || c >= R.ncell) break;
        const double4 g = R.cgeo[c];
        const double dx = g.x - x, dy = g.y - y, dz = g.z - z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (3.0 * (g.w * g.w) <= R.theta2 * d2) return point_expansion(dx, dy, dz, sc.x - g.x, sc.y - g.y, sc.z - g.z);
        const int link = R.cm[c].y;
        if (link < 0) {
            const double ex = x - sc.x, ey = y - sc.y, ez = z - sc.z;
            return rsqrt_nr(ex * ex + ey * ey + ez * ez);
        }
        if (link + 8 > R.ncell) break;
        c = link + key_digit(key, level + 1);
    }
    bad = 1;
    return 0.0;
}

// ------------------------------------------------------------ one Monte Carlo move
constexpr int kMaxPathCells = 4 * kMaxLevels;
constexpr int kLineContrib = 16;  // old and new position of up to 8 line images of the mover
constexpr int kPowCells = 24;  // longer path-cell lists build their monomials by repeated products
constexpr int kDrawBatch = 64;  // trial moves drawn ahead at once, one per lane of the first wave

struct McShared {
    int path[4][kMaxLevels];  // root paths: ion old, ion new, image old, image new
    double4 path_geo[4][kMaxLevels];  // geometry of each path cell, read with its link
    int plen[4];
    int fs0, level0;          // where the move traversal starts
    uint64_t key[4];
    double4 contrib[4];       // (position, charge) of the four contributions
    double alpha;             // the move's Metropolis uniform
    // commit state gathered while the traversal runs
    int2 tr[2];               // tracking (leaf cell, slot) of the ion and of its image
    int4 lm_old[2];           // (count, link, base, cap) of their leaves
    int4 lm_new[2];           // same for the leaves of their new positions
    int last_pidx[2];         // source in the last slot of each old leaf
    double4 last_pool[2];     // and its (x, y, z, q)
    int self_pidx[2];         // source found at the tracked slot (must be the mover)
    int pf_stage[2];
    // distinct cells of the four root paths with the contributions they take
    int nlist;
    int list_cell[kMaxPathCells];
    int list_mask[kMaxPathCells];   // bit jj: contribution jj applies; bit 4: internal cell
    double4 list_geo[kMaxPathCells];
    int ok;
    int err;
    int cnt2[2];
    // the next trial moves (index, dx, dy, dz, alpha), and the next mover's ion and image as
    // loaded while the current move's traversal runs
    int dr_i[kDrawBatch];
    double dr_d[kDrawBatch][4];
    double4 nx_si, nx_mo;
    // powers 0..p of each contribution's offset from each of the first kPowCells list cells,
    // per axis: d^n = x^n1 y^n2 z^n3 by two products
    double pw[kPowCells][4][3][P + 1];
    // the mover's line images (multiple-image model): old (2m) and new (2m + 1) position and
    // charge of line image m, the root paths of both, descended beside the traversal; for each
    // old one and each target the first path cell passing the MAC (level, or -1: its leaf sums
    // it directly; and its geometry); each new leaf's count and capacity
    double4 lpos[kLineContrib];
    double4 lmac_geo[kLineContrib / 2][2];
    uint64_t lkey[kLineContrib];
    int lpath[kLineContrib][kMaxLevels];
    int lplen[kLineContrib];
    int lmac[kLineContrib / 2][2];
    int lcnt[kLineContrib / 2], lcap[kLineContrib / 2];
    int lnext[kLineContrib];  // next level of each line path; -1 before its position is read
};

struct MoveOut { double dE; int reason; int accepted; int stop; int detail; };

constexpr double kInf = __builtin_huge_val();

// One stage of the commit prefetch for old source j (0: ion, 1: image).
__device__ __forceinline__ void prefetch_stage(const Rep& R, McShared& MS, int j, int s) {
    const int stage = MS.pf_stage[j];
    if (stage == 0) {
        const int2 t = gload(R.track + s);
        MS.tr[j] = t;
        MS.pf_stage[j] = (t.x >= 0 && t.x < R.ncell) ? 1 : 9;
    } else if (stage == 1) {
        const int4 m = gload(R.cm + MS.tr[j].x);
        MS.lm_old[j] = m;
        const bool sane = m.y < 0 && m.x >= 1 && m.z >= 0 && m.z + m.x <= R.pool && m.x <= m.w &&
                          MS.tr[j].y >= 0 && MS.tr[j].y < m.x;
        MS.pf_stage[j] = sane ? 2 : 9;
    } else if (stage == 2) {
        const int4 m = MS.lm_old[j];
        MS.last_pidx[j] = gload(R.pidx + m.z + m.x - 1);
        MS.last_pool[j] = gload(R.pool4 + m.z + m.x - 1);
        MS.self_pidx[j] = gload(R.pidx + m.z + MS.tr[j].y);
        MS.pf_stage[j] = 3;
    }
}

// ------------------------------------------------------------ line images of the mover
// The multiple-image model gives each ion M line-image sources (2n + m n + i) besides
// its Kelvin image.  A move keeps the mover's own line images in its traversal as
// ordinary sources.  Beside the traversal, lanes of an otherwise idle wave descend the
// root paths of their old and new positions (line_step), noting for each old one the
// first cell that passes the MAC for each target; afterwards each is taken back out of
// both potentials where the traversal met it (line_corrections), every leaf an accepted
// move fills is checked in commit order, and the line images are moved after the ion and
// its image, in source order, by the local modification of Sec. 3.3 (lines_commit).

// One step of line contribution j's root path (j = 2m: old position of line image m,
// 2m + 1: new), as the ion's own paths descend.
__device__ __forceinline__ void line_step(const Rep& R, McShared& MS, const double* tx, const double* ty,
                                          const double* tz, int j, int level, int i) {
    const int c = MS.lpath[j][level];
    const bool cok = c >= 0 && c < R.ncell;
    const bool old = (j & 1) == 0;
    int4 m = make_int4(0, -1, 0, 0);
    double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
    if (cok) {
        m = gload(R.cm + c);
        if (old) g = gload(R.cgeo + c);
    }
    if (!cok || (m.y >= 0 && m.y + 8 > R.ncell)) {
        MS.err = kErrPathCell;
        MS.lplen[j] = level + 1;
        MS.lpath[j][level] = 0;
        return;
    }
    if (old) {
        const int mm = j >> 1;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (MS.lmac[mm][t] >= 0) continue;
            const double dx = g.x - tx[t], dy = g.y - ty[t], dz = g.z - tz[t];
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (3.0 * (g.w * g.w) <= R.theta2 * d2) { MS.lmac[mm][t] = level; MS.lmac_geo[mm][t] = g; }
        }
    }
    if (m.y >= 0 && level + 1 < kMaxLevels) {
        MS.lpath[j][level + 1] = m.y + key_digit(MS.lkey[j], level + 1);
        return;
    }
    if (m.y >= 0) MS.err = kErrPathDepth;
    MS.lplen[j] = level + 1;
    if (!old) {
        MS.lcnt[j >> 1] = m.x;
        MS.lcap[j >> 1] = m.w;
        if (m.z < 0 || m.x < 0 || m.z + m.w > R.pool) MS.err = kErrCommitLeaf;
    } else if (gload(R.track + (2 * R.n + (j >> 1) * R.n + i)).x != c) {
        MS.err = kErrCommitSlot;  // the tracked leaf must be the one the old position's key leads to
    }
}

// Up to nsteps steps of line contribution j = tl's root path, its position read (old) or
// placed as the build places it from the new Kelvin image (new) on the first call.  The
// lane's state lives in LDS, so nothing of it stays in registers across the traversal.
__device__ __attribute__((noinline)) void line_lane_steps(const Rep& R, McShared& MS, const double* tx,
                                                          const double* ty, const double* tz, int tl, int i,
                                                          int nsteps) {
    int level = MS.lnext[tl];
    if (level < 0) {
        const int m = tl >> 1;
        double4 p;
        if (tl & 1) {
            const double4 k = MS.contrib[3];
            p = make_double4(R.line_t[m] * k.x, R.line_t[m] * k.y, R.line_t[m] * k.z, R.line_c[m] * k.w);
        } else {
            p = gload(R.src + (2 * R.n + m * R.n + i));
        }
        MS.lpos[tl] = p;
        MS.lkey[tl] = morton_key(R, p.x, p.y, p.z);
        level = 0;
    }
    for (int k = 0; k < nsteps && MS.lplen[tl] == 0 && level < kMaxLevels; ++k) line_step(R, MS, tx, ty, tz, tl, level++, i);
    MS.lnext[tl] = level;
}

// What the mover's own line images added to the potential at target t, from the paths
// descended beside the traversal: line image m through the expansion of the first cell of
// its root path that passes the MAC, else directly at its leaf.  Lanes 2m + t of every
// wave compute it, so each wave holds the sums without a barrier.
__device__ __attribute__((noinline)) void line_corrections(const Rep& R, const McShared& MS, double& c0, double& c1) {
    const int lane = lane_id(), t = lane & 1, m = lane >> 1;
    double v = 0.0;
    if (m < R.nline) {
        const double4 sc = MS.lpos[2 * m], x = MS.contrib[t];
        const int l = MS.lmac[m][t];
        if (l >= 0) {
            const double4 g = MS.lmac_geo[m][t];
            v = sc.w * point_expansion(g.x - x.x, g.y - x.y, g.z - x.z, sc.x - g.x, sc.y - g.y, sc.z - g.z);
        } else {
            const double ex = x.x - sc.x, ey = x.y - sc.y, ez = x.z - sc.z;
            v = sc.w * rsqrt_nr(ex * ex + ey * ey + ez * ez);
        }
    }
    c0 = wave_sum(t == 0 ? v : 0.0);
    c1 = wave_sum(t == 1 ? v : 0.0);
}

// Would the 2 + M insertions of this move (ion, Kelvin image, line images in source
// order) overflow a leaf?  Each new leaf is checked with the counts the earlier ones
// leave behind.
__device__ __forceinline__ int fit_old_leaf(const McShared& MS, int k) {
    return k == 0 ? MS.tr[0].x : (k == 1 ? MS.tr[1].x : MS.lpath[2 * (k - 2)][MS.lplen[2 * (k - 2)] - 1]);
}
__device__ __forceinline__ int fit_new_leaf(const McShared& MS, int k) {
    return k < 2 ? MS.path[2 * k + 1][MS.plen[2 * k + 1] - 1] : MS.lpath[2 * (k - 2) + 1][MS.lplen[2 * (k - 2) + 1] - 1];
}
__device__ __attribute__((noinline)) bool lines_fit(const Rep& R, const McShared& MS) {
    for (int k = 0; k < 2 + R.nline; ++k) {
        const int lo = fit_old_leaf(MS, k), ln = fit_new_leaf(MS, k);
        if (ln == lo) continue;
        int c = k < 2 ? MS.lm_new[k].x : MS.lcnt[k - 2];
        const int cap = k < 2 ? MS.lm_new[k].w : MS.lcap[k - 2];
        for (int e = 0; e < k; ++e) {
            const int eo = fit_old_leaf(MS, e), en = fit_new_leaf(MS, e);
            if (en == eo) continue;
            if (en == ln) c += 1;
            if (eo == ln) c -= 1;
        }
        if (c + 1 > cap) return false;
    }
    return true;
}

// Distinct cells of the 2M line paths, built in the frontier buffer (free after the
// traversal): bit j of a cell's mask = contribution j applies; kLineInternal = not a leaf.
struct LineList {
    int nlist;
    int cell[kLineContrib * kMaxLevels];
    uint32_t mask[kLineContrib * kMaxLevels];
};
constexpr uint32_t kLineInternal = 1u << 16;

template <int BLOCK>
__device__ __forceinline__ LineList& line_list(Trav<2, BLOCK>& S) {
    static_assert(sizeof(LineList) <= sizeof(S.front), "the line-path cell list must fit the frontier buffer");
    return *reinterpret_cast<LineList*>(&S.front[0][0]);
}

// Move one line image between leaf index arrays (or rewrite its slot) from the current
// state in HBM; false on a broken index.
__device__ __forceinline__ bool line_slot_move(const Rep& R, int s, int lo, int ln, double4 pn) {
    const int2 tr = R.track[s];
    const int4 mo = R.cm[lo];
    if (tr.x != lo || mo.y >= 0 || tr.y < 0 || tr.y >= mo.x || mo.z < 0 || mo.z + mo.x > R.pool) return false;
    if (ln != lo) {
        const int last = mo.x - 1, k = tr.y;
        const int4 mn = R.cm[ln];
        if (mn.y >= 0 || mn.x < 0 || mn.x + 1 > mn.w || mn.z < 0 || mn.z + mn.w > R.pool) return false;
        if (k != last) {
            const int moved = R.pidx[mo.z + last];
            if (moved < 0 || moved >= R.nsrc) return false;
            R.pool4[mo.z + k] = R.pool4[mo.z + last];
            R.pidx[mo.z + k] = moved;
            R.track[moved] = make_int2(lo, k);
        }
        R.cm[lo].x = last;
        R.pool4[mn.z + mn.x] = pn;
        R.pidx[mn.z + mn.x] = s;
        R.track[s] = make_int2(ln, mn.x);
        R.cm[ln].x = mn.x + 1;
    } else {
        R.pool4[mo.z + tr.y] = pn;
    }
    R.src[s] = pn;
    return true;
}

// After the ion and its image: the line images' slot moves (one lane each when no two
// of them touch a common leaf, else one lane in source order), beside them the distinct
// cells of their 2M root paths, then every thread repairs those cells' moments and counts,
// applying to each cell, in order, old line image 0 (-), new line image 0 (+), old 1 ...
// LL.nlist must be 0 on entry.
template <int BLOCK>
__device__ __forceinline__ void lines_commit(const Rep& R, Trav<2, BLOCK>& S, McShared& MS, int i) {
    LineList& LL = line_list(S);
    const int tid = threadIdx.x, M = R.nline, nc = 2 * M;
    if (wave_id() == 0) {
        const int m = lane_id();
        int lo = -1, ln = -1;
        if (m < M) {
            lo = MS.lpath[2 * m][MS.lplen[2 * m] - 1];
            ln = MS.lpath[2 * m + 1][MS.lplen[2 * m + 1] - 1];
        }
        bool clash = false;
        for (int e = 0; e < M; ++e) {
            const int eo = __shfl(lo, e, 64), en = __shfl(ln, e, 64);
            if (m < M && e != m && (eo == lo || eo == ln || en == lo || en == ln)) clash = true;
        }
        if (__ballot(clash) == 0) {
            if (m < M && !line_slot_move(R, 2 * R.n + m * R.n + i, lo, ln, MS.lpos[2 * m + 1])) MS.err = kErrCommitSlot;
        } else if (m == 0) {
            for (int k = 0; k < M; ++k) {
                const int ko = MS.lpath[2 * k][MS.lplen[2 * k] - 1], kn = MS.lpath[2 * k + 1][MS.lplen[2 * k + 1] - 1];
                if (!line_slot_move(R, 2 * R.n + k * R.n + i, ko, kn, MS.lpos[2 * k + 1])) { MS.err = kErrCommitSlot; break; }
            }
        }
    } else {
        for (int it = tid - 64; it < nc * kMaxLevels; it += BLOCK - 64) {
            const int j = it / kMaxLevels, l = it % kMaxLevels;
            if (l >= MS.lplen[j]) continue;
            const int c = MS.lpath[j][l];
            bool owner = true;
            for (int jj = 0; jj < j; ++jj)
                if (l < MS.lplen[jj] && MS.lpath[jj][l] == c) owner = false;
            if (!owner) continue;
            uint32_t mask = l < MS.lplen[j] - 1 ? kLineInternal : 0u;
            for (int jj = j; jj < nc; ++jj)
                if (l < MS.lplen[jj] && MS.lpath[jj][l] == c) mask |= 1u << jj;
            const int slot = atomicAdd(&LL.nlist, 1);
            LL.cell[slot] = c;
            LL.mask[slot] = mask;
        }
    }
    __syncthreads();
    const int items = LL.nlist * NTERM;
    for (int it = tid; it < items; it += BLOCK) {
        const int li = it / NTERM, k = it % NTERM;
        const int c = LL.cell[li];
        const uint32_t mask = LL.mask[li];
        const double4 g = R.cgeo[c];
        double mk = R.M[(size_t)c * MSTR + k];
        int dc = 0;
        for (int j = 0; j < nc; ++j) {
            if (!(mask & (1u << j))) continue;
            const double4 sp = MS.lpos[j];
            const double v = mono(S.mi[k], sp.x - g.x, sp.y - g.y, sp.z - g.z);
            if (j & 1) { mk = mk + sp.w * v; ++dc; } else { mk = mk - sp.w * v; --dc; }
        }
        R.M[(size_t)c * MSTR + k] = mk;
        if (R.M32) R.M32[(size_t)c * MSTR + k] = (float)mk;
        if (k == 0 && (mask & kLineInternal) && dc != 0) R.cm[c].x += dc;
    }
    __syncthreads();
}

// Local modification of Sec. 3.3 for an accepted move.  Thread 0 moves the
// ion and then its image between leaf index arrays (delete = the last entry
// fills the hole; add = append) from the state gathered during the
// traversal; the other threads repair the moments and counts of the distinct
// cells of the four root paths, applying to each cell, in order, the old ion
// (-), the new ion (+), the old image (-) and the new image (+).
template <int BLOCK>
__device__ __forceinline__ void commit(const Rep& R, const Trav<2, BLOCK>& S, McShared& MS, int i) {
    const int tid = threadIdx.x;
    const bool imgs = R.images != 0;
    const bool use_pw = MS.nlist <= kPowCells;
    if (use_pw) {
        for (int it = tid; it < MS.nlist * 12; it += BLOCK) {
            const int li = it / 12, r = it % 12, jj = r / 3, ax = r % 3;
            const double4 s = MS.contrib[jj], g = MS.list_geo[li];
            const double d = ax == 0 ? s.x - g.x : (ax == 1 ? s.y - g.y : s.z - g.z);
            double v = 1.0;
            MS.pw[li][jj][ax][0] = 1.0;
            for (int e = 1; e <= P; ++e) { v *= d; MS.pw[li][jj][ax][e] = v; }
        }
        __syncthreads();
    }
    if (tid == 0) {
        // leaf states: cell, base, count of up to four leaves, followed through the moves
        int lc[4], lb[4], ln[4];
        int nl = 0;
        auto find = [&](int cell, int base, int count) {
            for (int k = 0; k < nl; ++k)
                if (lc[k] == cell) return k;
            lc[nl] = cell; lb[nl] = base; ln[nl] = count;
            return nl++;
        };
        const int a = find(MS.tr[0].x, MS.lm_old[0].z, MS.lm_old[0].x);
        const int b = find(MS.path[1][MS.plen[1] - 1], MS.lm_new[0].z, MS.lm_new[0].x);
        int img_slot = imgs ? MS.tr[1].y : -1;
        const int K = R.n + i;
        const double4 ion_new = MS.contrib[1];
        if (a != b) {
            const int k = MS.tr[0].y, last = ln[a] - 1;
            const int moved = MS.last_pidx[0];
            if (k != last) {
                R.pool4[lb[a] + k] = MS.last_pool[0];
                R.pidx[lb[a] + k] = moved;
                if (moved >= 0 && moved < R.nsrc) R.track[moved] = make_int2(lc[a], k);
                else MS.err = kErrCommitSource;
                if (moved == K) img_slot = k;
            }
            ln[a] = last;
            R.cm[lc[a]].x = last;
            const int pos = ln[b];
            R.pool4[lb[b] + pos] = ion_new;
            R.pidx[lb[b] + pos] = i;
            R.track[i] = make_int2(lc[b], pos);
            ln[b] = pos + 1;
            R.cm[lc[b]].x = pos + 1;
        } else {
            R.pool4[lb[a] + MS.tr[0].y] = ion_new;
        }
        R.src[i] = ion_new;
        if (imgs) {
            const int c_old = MS.tr[1].x;
            const int touched = (c_old == lc[a] || c_old == lc[b]);
            const int cc = find(c_old, MS.lm_old[1].z, MS.lm_old[1].x);
            const int dd = find(MS.path[3][MS.plen[3] - 1], MS.lm_new[1].z, MS.lm_new[1].x);
            const double4 img_new = MS.contrib[3];
            if (cc != dd) {
                const int last = ln[cc] - 1;
                int moved;
                double4 mv;
                if (!touched) {
                    moved = MS.last_pidx[1];
                    mv = MS.last_pool[1];
                } else {  // the ion's move changed this leaf: read its last entry again
                    moved = R.pidx[lb[cc] + last];
                    mv = R.pool4[lb[cc] + last];
                }
                if (img_slot != last) {
                    R.pool4[lb[cc] + img_slot] = mv;
                    R.pidx[lb[cc] + img_slot] = moved;
                    if (moved >= 0 && moved < R.nsrc) R.track[moved] = make_int2(lc[cc], img_slot);
                    else MS.err = kErrCommitSource;
                }
                ln[cc] = last;
                R.cm[lc[cc]].x = last;
                const int pos = ln[dd];
                R.pool4[lb[dd] + pos] = img_new;
                R.pidx[lb[dd] + pos] = K;
                R.track[K] = make_int2(lc[dd], pos);
                ln[dd] = pos + 1;
                R.cm[lc[dd]].x = pos + 1;
            } else {
                R.pool4[lb[cc] + img_slot] = img_new;
            }
            R.src[K] = img_new;
        }
    }
    // moments and counts of the distinct path cells: all loads first, then stores
    const int items = MS.nlist * NTERM;
    constexpr int G = 4;
    for (int base = tid; base < items; base += G * BLOCK) {
        double mk[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int it = base + u * BLOCK;
            if (it < items) {
                const int li = it / NTERM, k = it % NTERM;
                mk[u] = R.M[(size_t)MS.list_cell[li] * MSTR + k];
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int it = base + u * BLOCK;
            if (it >= items) continue;
            const int li = it / NTERM, k = it % NTERM;
            const int c = MS.list_cell[li], mask = MS.list_mask[li];
            const double4 g = MS.list_geo[li];
            double m = mk[u];
            int dc = 0;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                if (!(mask & (1 << jj))) continue;
                const double4 s = MS.contrib[jj];
                double v;
                if (use_pw) {
                    const uint32_t code = S.mi[k];
                    v = MS.pw[li][jj][0][code & 255u] * MS.pw[li][jj][1][(code >> 8) & 255u] *
                        MS.pw[li][jj][2][code >> 16];
                } else {
                    v = mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z);
                }
                if (jj & 1) { m = m + s.w * v; ++dc; } else { m = m - s.w * v; --dc; }
            }
            R.M[(size_t)c * MSTR + k] = m;
            if (R.M32) R.M32[(size_t)c * MSTR + k] = (float)m;
            if (k == 0 && (mask & 16) && dc != 0) R.cm[c].x += dc;
        }
    }
    __syncthreads();
}

// mode 0: evaluate; 1: Metropolis with alpha, commit if accepted;
// 2: commit unless rejected by a wall or an overlap.
//
// si and mo are the mover's ion and image as stored (mo unused without images);
// inext >= 0 names the next move's ion, whose sources one lane loads into
// MS.nx_si / MS.nx_mo during the traversal (valid if the ion is not i).
template <int BLOCK, bool LINES>
__device__ __forceinline__ MoveOut one_move(const Rep& R, Trav<2, BLOCK>& S, McShared& MS, int i, double4 si,
                            double4 mo, double rx, double ry, double rz, double alpha, int mode, int inext) {
    static_assert(BLOCK >= 256, "the path descents, the commit prefetch and the next mover's load run on "
                                "the last three waves");
    const int tid = threadIdx.x;
    MoveOut out{kInf, 0, 0, 0, 0};
    const bool imgs = R.images != 0;
    const int nps = imgs ? 4 : 2;
    if (outside(R, rx, ry, rz)) { out.reason = 1; return out; }
    if (tid < 4) {
        // lane j sets up contribution j (old ion, new ion, old image, new image) and its key,
        // the four side by side; lane 0 then writes the targets' state
        const int j = tid;
        double4 cj;
        if (j == 0) cj = si;
        else if (j == 1) cj = make_double4(rx, ry, rz, si.w);
        else if (j == 2) cj = mo;
        else cj = imgs ? kelvin(R, rx, ry, rz, si.w) : make_double4(0, 0, 0, 0);
        const uint64_t kj = (j < 2 || imgs) ? morton_key(R, cj.x, cj.y, cj.z) : 0;
        MS.key[j] = kj;
        MS.contrib[j] = cj;
        const uint32_t klo = (uint32_t)kj, khi = (uint32_t)(kj >> 32);
        const uint64_t kio = (uint64_t)(uint32_t)__shfl((int)klo, 0, 64) |
                             ((uint64_t)(uint32_t)__shfl((int)khi, 0, 64) << 32);
        const uint64_t kmo = (uint64_t)(uint32_t)__shfl((int)klo, 2, 64) |
                             ((uint64_t)(uint32_t)__shfl((int)khi, 2, 64) << 32);
        if (j == 0) {
            S.tx[0] = si.x; S.ty[0] = si.y; S.tz[0] = si.z;
            S.tx[1] = rx; S.ty[1] = ry; S.tz[1] = rz;
            for (int t = 0; t < 2; ++t) {
                S.ex_i[t] = i; S.ex_k[t] = imgs ? R.n + i : -1;
                S.kx_i[t] = kio; S.kx_k[t] = kmo;
                S.es_i[t] = si; S.es_k[t] = mo;
            }
            S.ovl_t = 1; S.ovl_ex = i; S.n_ovl = 0;
            S.err = 0; S.overlap = 0; S.coincide = 0;
            // The root holds both targets, so the MAC never takes it (theta < 1): it is opened
            // for both whenever it is split and holds more than N_0 sources besides the two
            // excluded ones.  Then the traversal starts from its children, cells 1..8 in digit
            // order.
            const int np_root = R.nsrc - 1 - (imgs ? 1 : 0);
            if (R.ncell > 1 && np_root > R.n0) {
                const int di = key_digit(kio, 1), dk = imgs ? key_digit(kmo, 1) : -1;
                for (int d = 0; d < 8; ++d)
                    S.front[0][d] = (uint32_t)(1 + d) | (3u << kMaskSh) | (d == di ? kFlagIon : 0u) |
                                    (d == dk ? kFlagImg : 0u);
                MS.fs0 = 8;
                MS.level0 = 1;
            } else {
                S.front[0][0] = (3u << kMaskSh) | kFlagIon | (imgs ? kFlagImg : 0u);
                MS.fs0 = 1;
                MS.level0 = 0;
            }
            MS.alpha = alpha;
            MS.err = 0;
            MS.nlist = 0;
        }
    }
    // work beside the traversal runs on the last waves, which have no frontier entries to
    // classify on most levels, each task on a wave of its own (divergent lanes of one wave
    // would wait for their loads one after another): the root-path descents on lanes 0-3 of
    // the last wave, the commit prefetch on lanes 0-1 of the wave before it, and the next
    // mover's load on lane 0 of the wave before that
    const int th = tid - (BLOCK - 64), tp = tid - (BLOCK - 128);
    if (th >= 0 && th < 4) { MS.path[th][0] = 0; MS.plen[th] = 0; }
    if (tp == 0 || tp == 1) MS.pf_stage[tp] = (tp == 1 && !imgs) ? 3 : 0;
    int my_level = 0;  // the next level of this lane's root path
    // the line images' root paths (multiple-image model) on lanes 16 .. 16 + 2M - 1 of the
    // wave that loads the next mover
    {
        const int tl = tid - (BLOCK - 192) - 16;
        if (LINES && tl >= 0 && tl < 2 * R.nline) {
            MS.lpath[tl][0] = 0;
            MS.lplen[tl] = 0;
            MS.lnext[tl] = -1;
            if (!(tl & 1)) { MS.lmac[tl >> 1][0] = -1; MS.lmac[tl >> 1][1] = -1; }
        }
    }
    __syncthreads();
    // one step of a root path: descend by the key's digit, or stop at the leaf
    auto step = [&](int pj, int level) {
        const int c = MS.path[pj][level];
        const bool cok = c >= 0 && c < R.ncell;
        const int link = cok ? gload(R.cm + c).y : -1;
        if (cok) MS.path_geo[pj][level] = gload(R.cgeo + c);
        if (c < 0 || c >= R.ncell || (link >= 0 && link + 8 > R.ncell)) {
            MS.err = kErrPathCell;
            MS.plen[pj] = level + 1;
            MS.path[pj][level] = 0;
        } else if (link >= 0 && level + 1 < kMaxLevels) {
            MS.path[pj][level + 1] = link + key_digit(MS.key[pj], level + 1);
        } else {
            if (link >= 0) MS.err = kErrPathDepth;
            MS.plen[pj] = level + 1;
            if (pj & 1) {  // a new position's leaf: its slot state for the commit
                const int4 m = gload(R.cm + c);
                MS.lm_new[pj >> 1] = m;
                if (m.y >= 0 || m.z < 0 || m.x < 0 || m.z + m.w > R.pool) MS.err = kErrCommitLeaf;
            }
        }
    };
    // the root paths descend two levels, and the commit state two stages, per traversal level;
    // the next mover's sources are loaded on the first level
    auto hook = [&](int level) {
        if (th >= 0 && th < nps)
            for (int k = 0; k < 2 && MS.plen[th] == 0 && my_level < kMaxLevels; ++k) step(th, my_level++);
        if (tp == 0 || tp == 1)
            for (int k = 0; k < 2; ++k) prefetch_stage(R, MS, tp, tp == 0 ? i : R.n + i);
        if (tp == -64 && level == MS.level0 && inext >= 0) {
            MS.nx_si = R.src[inext];
            MS.nx_mo = imgs ? R.src[R.n + inext] : make_double4(0, 0, 0, 0);
        }
        if (LINES && tid - (BLOCK - 192) - 16 >= 0 && tid - (BLOCK - 192) - 16 < 2 * R.nline)
            line_lane_steps(R, MS, S.tx, S.ty, S.tz, tid - (BLOCK - 192) - 16, i, 2);
    };
    double pot[2];
    const int levels = traverse_mc<BLOCK>(R, S, MS.cnt2, hook, MS.fs0, MS.level0, pot);
    (void)levels;
    if (S.err) {
        out.stop = (S.err == kErrStack || S.err == kErrFrontier) ? -7 : -8;
        out.detail = S.err;
        __syncthreads();
        return out;
    }
    if (th >= 0 && th < nps) {
        while (MS.plen[th] == 0 && my_level < kMaxLevels) step(th, my_level++);
        if (MS.plen[th] == 0) { MS.err = kErrPathDepth; MS.plen[th] = 1; MS.path[th][0] = 0; }
    }
    if (tp == 0 || tp == 1) {
        const int s = tp == 0 ? i : R.n + i;
        for (int k = 0; k < 3 && MS.pf_stage[tp] < 3; ++k) prefetch_stage(R, MS, tp, s);
        if (MS.pf_stage[tp] != 3) MS.err = kErrCommitSlot;
    }
    {
        const int tl = tid - (BLOCK - 192) - 16;
        if (LINES && tl >= 0 && tl < 2 * R.nline) {
            line_lane_steps(R, MS, S.tx, S.ty, S.tz, tl, i, kMaxLevels);
            if (MS.lplen[tl] == 0) { MS.err = kErrPathDepth; MS.lplen[tl] = 1; MS.lpath[tl][0] = 0; }
        }
    }
    __syncthreads();
    if (MS.err) { out.stop = -8; out.detail = MS.err; __syncthreads(); return out; }
    // distinct cells of the root paths (any order: each cell's updates are applied by one thread set)
    for (int it = tid; it < nps * kMaxLevels; it += BLOCK) {
        const int j = it / kMaxLevels, l = it % kMaxLevels;
        if (l >= MS.plen[j]) continue;
        const int c = MS.path[j][l];
        bool owner = true;
        for (int jj = 0; jj < j; ++jj)
            if (l < MS.plen[jj] && MS.path[jj][l] == c) owner = false;
        if (!owner) continue;
        int mask = l < MS.plen[j] - 1 ? 16 : 0;
        for (int jj = j; jj < nps; ++jj)
            if (l < MS.plen[jj] && MS.path[jj][l] == c) mask |= 1 << jj;
        const int slot = atomicAdd(&MS.nlist, 1);
        MS.list_cell[slot] = c;
        MS.list_mask[slot] = mask;
        MS.list_geo[slot] = MS.path_geo[j][l];
    }
    const double po = pot[0], pn = pot[1];
    if (S.overlap || S.coincide) { out.reason = 2; __syncthreads(); return out; }
    double lc0 = 0.0, lc1 = 0.0;  // what the mover's own line images added at the two targets
    if (LINES && R.nline > 0) line_corrections(R, MS, lc0, lc1);
    // the move's positions and alpha come back from LDS: no registers held across the traversal
    const double4 so = MS.contrib[0], sn = MS.contrib[1];
    const double q = so.w, l = R.l_B;
    double dE = LINES && R.nline > 0 ? l * q * ((pn - lc1) - (po - lc0)) : l * q * (pn - po);
    if (R.geom == 1) {
        const double rn2 = sn.x * sn.x + sn.y * sn.y + sn.z * sn.z;
        const double ro2 = so.x * so.x + so.y * so.y + so.z * so.z;
        if (imgs) dE += 0.5 * l * R.gamma * R.a * q * q * (1.0 / (rn2 - R.a2) - 1.0 / (ro2 - R.a2));
        // own line images: c_m q_K at t_m r_K, |r - t_m r_K| = (r^2 - t_m a^2) / |r|
        if (LINES)
            for (int m = 0; m < R.nline; ++m)
                dE += 0.5 * l * R.line_c[m] * R.gamma * R.a * q * q *
                      (1.0 / (rn2 - R.line_t[m] * R.a2) - 1.0 / (ro2 - R.line_t[m] * R.a2));
        if (R.Qc != 0.0) dE += l * R.Qc * q * (1.0 / sqrt(rn2) - 1.0 / sqrt(ro2));
    }
    out.dE = dE;
    bool acc = false;
    if (mode == 1) acc = dE <= 0.0 || MS.alpha <= exp(-dE);
    else if (mode == 2) acc = true;
    if (!acc) { __syncthreads(); return out; }
    if (tid == BLOCK - 1) {  // a thread with no path-cell item above
        // the tracked leaves must be the leaves the old positions' keys lead to,
        // and the tracked slots must hold the movers
        bool sane = MS.tr[0].x == MS.path[0][MS.plen[0] - 1] && MS.self_pidx[0] == i;
        if (imgs) sane = sane && MS.tr[1].x == MS.path[2][MS.plen[2] - 1] && MS.self_pidx[1] == R.n + i;
        sane = sane && MS.last_pidx[0] >= 0 && MS.last_pidx[0] < R.nsrc;
        bool ok = sane;
        if (sane) {
            const int cio = MS.tr[0].x, cin = MS.path[1][MS.plen[1] - 1];
            if (cin != cio && MS.lm_new[0].x + 1 > MS.lm_new[0].w) ok = false;
            if (imgs) {
                const int cmo = MS.tr[1].x, cmn = MS.path[3][MS.plen[3] - 1];
                if (cmn != cmo) {
                    int c = MS.lm_new[1].x;
                    if (cin != cio) { if (cmn == cin) c += 1; if (cmn == cio) c -= 1; }
                    if (c + 1 > MS.lm_new[1].w) ok = false;
                }
            }
        } else {
            MS.err = kErrCommitSlot;
        }
        if (LINES && R.nline > 0) {
            if (ok && !lines_fit(R, MS)) ok = false;  // every insertion of the move, in commit order
            line_list(S).nlist = 0;
        }
        MS.ok = ok;
    }
    __syncthreads();
    if (MS.err) { out.stop = -8; out.detail = MS.err; __syncthreads(); return out; }
    if (!MS.ok) { out.stop = -6; __syncthreads(); return out; }
    commit<BLOCK>(R, S, MS, i);
    if (LINES && R.nline > 0 && !MS.err) lines_commit<BLOCK>(R, S, MS, i);
    if (MS.err) { out.stop = -8; out.detail = MS.err; }
    out.accepted = 1;
    return out;
}

// ------------------------------------------------------------ kernels
constexpr int kMcBlock = 512;      // a single chain: the widest traversal per move
constexpr int kMcBlockBatch = 256; // replicas: two workgroups per CU hide each other's latency
constexpr int kEnergyBlock = 256;
constexpr int kEnergyTargets = 4;

__device__ __forceinline__ void load_rep(Rep& dst, const Rep* src) {
    constexpr int W = (int)(sizeof(Rep) / 8);
    static_assert(sizeof(Rep) % 8 == 0, "Rep is copied as 8-byte words");
    const uint64_t* a = (const uint64_t*)src;
    uint64_t* b = (uint64_t*)&dst;
    for (int k = threadIdx.x; k < W; k += blockDim.x) b[k] = a[k];
}

// Persistent Metropolis kernel: each workgroup takes replicas from the queue
// and advances its chain from move_next to move_end (Sec. 2 steps 1-3 with the
// treecode energy change and the local adjustment of Sec. 3.3).  A replica
// whose accepted move would overflow a leaf index array stops before that
// move with mc_status = ECAPACITY; the host rebuilds it and resumes.
template <int BLOCK, bool LINES>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_mc(Rep* reps, McArgs A) {
    __shared__ Trav<2, BLOCK> S;
    __shared__ McShared MS;
    __shared__ Rep Rs;
    __shared__ int s_r;
    const int tid = threadIdx.x;
    fill_mi(S);  // published by the first barrier below
    for (;;) {
        if (tid == 0) {
            const int qi = atomicAdd(A.queue, 1);
            s_r = qi < A.nlist ? A.list[qi] : -1;
        }
        __syncthreads();
        const int r = s_r;
        if (r < 0) break;
        load_rep(Rs, reps + r);
        __syncthreads();
        long long m = Rs.move_next;
        const long long m0 = m, mend = Rs.move_end;
        const bool imgs = Rs.images != 0;
        long long st_moves = 0, st_acc = 0, st_wall = 0, st_ovl = 0, st_met = 0;
        int status = 0, detail = 0;
        int prev_i = -1;
        bool have_nx = false;  // MS.nx_si / nx_mo hold this move's sources as of the last move
        for (; m < mend; ++m) {
            const int b = (int)((m - m0) & (kDrawBatch - 1));
            if (b == 0) {
                // the first wave draws the next kDrawBatch moves, one per lane
                if (tid < kDrawBatch && m + tid < mend) {
                    const Draw d = draw_move(A.seed, (uint32_t)r, (uint64_t)(m + tid), Rs.n, A.step);
                    MS.dr_i[tid] = d.i;
                    MS.dr_d[tid][0] = d.dx; MS.dr_d[tid][1] = d.dy; MS.dr_d[tid][2] = d.dz;
                    MS.dr_d[tid][3] = d.alpha;
                }
                __syncthreads();
            }
            const int i = MS.dr_i[b];
            const int inext = (b + 1 < kDrawBatch && m + 1 < mend) ? MS.dr_i[b + 1] : -1;
            // the last move changed only its own ion and image
            const bool use_nx = have_nx && i != prev_i;
            const double4 si = use_nx ? MS.nx_si : Rs.src[i];
            const double4 mo = use_nx ? MS.nx_mo : (imgs ? Rs.src[Rs.n + i] : make_double4(0, 0, 0, 0));
            const MoveOut o = one_move<BLOCK, LINES>(Rs, S, MS, i, si, mo, si.x + MS.dr_d[b][0], si.y + MS.dr_d[b][1],
                                              si.z + MS.dr_d[b][2], MS.dr_d[b][3], 1, inext);
            // a move outside the walls returns before its traversal, so before the load
            have_nx = inext >= 0 && o.reason != 1;
            prev_i = i;
            if (o.stop) { status = o.stop; detail = o.detail; break; }
            ++st_moves;
            if (o.accepted) ++st_acc;
            else if (o.reason == 1) ++st_wall;
            else if (o.reason == 2) ++st_ovl;
            else ++st_met;
            if (A.accept && tid == 0) A.accept[m - A.move_base] = (uint8_t)o.accepted;
            __syncthreads();
        }
        if (tid == 0) {
            Rep* g = reps + r;
            g->move_next = m;
            g->mc_status = status;
            if (detail) g->err_detail = detail;
            g->stats[0] += st_moves; g->stats[1] += st_acc; g->stats[2] += st_wall;
            g->stats[3] += st_ovl; g->stats[4] += st_met;
        }
        __syncthreads();
    }
}

template <bool LINES>
__global__ void __launch_bounds__(kMcBlock) k_move(Rep* reps, int r, MoveIO* io) {
    __shared__ Trav<2, kMcBlock> S;
    __shared__ McShared MS;
    __shared__ Rep Rs;
    fill_mi(S);
    load_rep(Rs, reps + r);
    __syncthreads();
    const int i = io->i;
    const double4 si = Rs.src[i];
    const double4 mo = Rs.images ? Rs.src[Rs.n + i] : make_double4(0, 0, 0, 0);
    const MoveOut o = one_move<kMcBlock, LINES>(Rs, S, MS, i, si, mo, io->rn[0], io->rn[1], io->rn[2], 0.0,
                                         io->mode == 0 ? 0 : 2, -1);
    if (threadIdx.x == 0) {
        io->dE = o.dE;
        io->reason = o.reason;
        io->status = o.stop;
        if (o.detail) reps[r].err_detail = o.detail;
    }
}

#include "bhmc_moves.hpp"

// Potential at every ion, with the ion and its image excluded, and each ion's term of
//   E / l_B = 1/2 q phi + 1/2 gamma a q^2 / (r^2 - a^2) + Q q / r.
// A workgroup takes kEnergyTargets consecutive positions of the build's key
// order (a space-filling curve) and traverses for the ions among them, so that
// its targets are close in space and share most of their interaction lists.
__global__ void __launch_bounds__(kEnergyBlock) k_energy(Rep* reps, int r, double* phi, double* eterm) {
    constexpr int NTG = kEnergyTargets;
    __shared__ Trav<NTG, kEnergyBlock> S;
    __shared__ Rep Rs;
    __shared__ int cnt2[2];
    __shared__ int s_ion[NTG];
    __shared__ int s_nv;
    fill_mi(S);
    load_rep(Rs, reps + r);
    __syncthreads();
    const int tid = threadIdx.x;
    const bool imgs = Rs.images != 0;
    const int ngroups = (Rs.nsrc + NTG - 1) / NTG;
    // one group of positions per workgroup, or several when the grid is bounded (HBM frontier regions)
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int k0 = grp * NTG;
        if (tid == 0) {
            int nv = 0;
            for (int j = 0; j < NTG && k0 + j < Rs.nsrc; ++j) {
                const int sid = Rs.perm[k0 + j];
                if ((unsigned)sid < (unsigned)Rs.n) s_ion[nv++] = sid;
            }
            s_nv = nv;
        }
        __syncthreads();
        const int nv = s_nv;
        if (nv == 0) {  // uniform: only images at these positions
            __syncthreads();
            continue;
        }
        if (tid < nv) {
            const int ion = s_ion[tid];
            const double4 si = Rs.src[ion];
            const double4 mo = imgs ? Rs.src[Rs.n + ion] : make_double4(0, 0, 0, 0);
            S.tx[tid] = si.x; S.ty[tid] = si.y; S.tz[tid] = si.z;
            S.ex_i[tid] = ion; S.ex_k[tid] = imgs ? Rs.n + ion : -1;
            S.kx_i[tid] = morton_key(Rs, si.x, si.y, si.z);
            S.kx_k[tid] = imgs ? morton_key(Rs, mo.x, mo.y, mo.z) : 0;
            S.es_i[tid] = si; S.es_k[tid] = mo;
            S.front[0][tid] = pack(0, tid, kFlagIon | (imgs ? kFlagImg : 0u));
        }
        if (tid == 0) { S.ovl_t = -1; S.ovl_ex = -1; S.n_ovl = 0; S.err = 0; S.overlap = 0; S.coincide = 0; }
        __syncthreads();
        traverse<NTG, kEnergyBlock>(Rs, S, nv, cnt2, [](int) {});
        if (tid < nv) {
            const int ion = s_ion[tid];
            const double4 si = Rs.src[ion];
            const double ph = S.err ? __builtin_nan("") : S.res[tid];
            if (S.err && tid == 0) reps[r].err_detail = S.err;
            double e = 0.5 * si.w * ph;
            if (Rs.geom == 1) {
                const double r2 = si.x * si.x + si.y * si.y + si.z * si.z;
                if (imgs) e += 0.5 * Rs.gamma * Rs.a * si.w * si.w / (r2 - Rs.a2);
                if (Rs.Qc != 0.0) e += Rs.Qc * si.w / sqrt(r2);
            }
            if (phi) phi[ion] = ph;
            eterm[ion] = e;
        }
        __syncthreads();  // the next group reuses the traversal state
    }
}

// Gradient of the treecode energy, step 1.  The ions, in the order of the
// build's key sort, are cut into groups of 16; one workgroup
// takes a group as the targets of one shared traversal: a frontier entry is a
// cell with four 16-bit masks (targets for which the cell is still open,
// targets summing every source below it directly (the N_0 rule), targets
// whose own image lies inside the cell, targets whose own ion does).  Each
// target takes exactly the decisions its own traversal would take (Sec. 3.2),
// so the interaction lists are the same.
// Far cells and near leaves are then evaluated by 16-lane rows with lane k
// serving target k: a row evaluates one far cell for all its targets, giving
// each the potential P and the field F_k = sum_m m_k T_m M^{m - e_k} (T up
// to order p + 1), and sums the targets' adjoint coefficients w T_n across the
// row before one device atomic per term; a near leaf is walked source by
// source, each pair's source side summed across the row before it is added
// to G.  The far cell that holds a target's own image is corrected afterwards
// (its pair terms with the image are taken out of P, F and G).  Per target:
//   dE/dx_t += -1/2 l_B q_t F_t,   dE/dq_t += 1/2 l_B P_t,
// and eterm gets the ion's energy term as in k_energy.
constexpr int kGradBlock = 256;
constexpr int kGradRows = kGradBlock / 16;
constexpr int kGT = 16;

struct GradShared {
    static constexpr int FCAP = 2048;  // on chip; larger levels continue in the HBM regions
    static constexpr int FARCAP = 512 + kGradBlock;
    static constexpr int NEARCAP = 256 + kGradBlock;
    static constexpr int NW = kGradBlock / 64;
    // first in the block, so that every term's LDS address is a row base plus an
    // immediate offset below 64 KiB (no per-term address registers)
    union {
        double mrow[kGradRows][MSTR];        // the moment rows of the far cells of one step, one per row
        double red[kGradRows][kGT][4];       // the rows' sums of each target at the end
    };
    uint32_t fc[2][FCAP];          // cell
    uint64_t fm[2][FCAP];          // open | direct << 16 | image inside << 32 | ion inside << 48
    uint32_t farc[FARCAP], farm[FARCAP];
    uint32_t nearc[NEARCAP], nearm[NEARCAP];
    double tx[kGT], ty[kGT], tz[kGT], tq[kGT];
    int ion[kGT];
    uint64_t kimg[kGT], kion[kGT];
    int flag_cell[kGT];
    int nt;
    uint64_t wcnt[2][NW];
    int err;
};

// A double read from another lane of the same 16-lane row by a DPP control
// (two 32-bit moves), no memory traffic; every control used here has a source
// lane inside the row for every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Reduce-scatter over the 16 lanes of a row: before, every lane holds x[0..15];
// after, x[0] of lane l holds the row's sum of x[i(l)], with
// i(l) = b3 << 3 | (b0 ^ b2) << 2 | (b1 ^ b2) << 1 | b2 for the bits b_j of l in
// its row.  Four exchange stages with the partners l ^ 8, l ^ 1, l ^ 2 and
// l ^ 7 (DPP row_ror:8, two quad permutations, row_half_mirror); at each stage
// a lane keeps the half of its values that its partner does not keep and adds
// the partner's copy of that half.  15 exchanges instead of the 64 of sixteen
// row sums, and every lane ends with a distinct index.
template <int CTRL, int M>
__device__ __forceinline__ void rs_stage(double (&x)[16], bool up) {
#pragma unroll
    for (int j = 0; j < M / 2; ++j) {
        const double lo = x[j], hi = x[j + M / 2];
        x[j] = (up ? hi : lo) + dpp_f64<CTRL>(up ? lo : hi);
    }
}
__device__ __forceinline__ int rs_index(int l) {
    return (((l >> 3) & 1) << 3) | (((l ^ (l >> 2)) & 1) << 2) | ((((l >> 1) ^ (l >> 2)) & 1) << 1) | ((l >> 2) & 1);
}
__device__ __forceinline__ double row_reduce_scatter16(double (&x)[16], int l) {
    rs_stage<0x128, 16>(x, (l >> 3) & 1);
    rs_stage<0xB1, 8>(x, (l ^ (l >> 2)) & 1);
    rs_stage<0x4E, 4>(x, ((l >> 1) ^ (l >> 2)) & 1);
    rs_stage<0x141, 2>(x, (l >> 2) & 1);
    return x[0];
}
// Row sums of four values by the first two stages above and two plain sums:
// every lane gets the sum of value b3 << 1 | (b0 ^ b2), so lanes 0, 1, 8 and 9
// of the row hold the sums of a, b, c and d.
__device__ __forceinline__ double row_sum4_scatter(double a, double b, double c, double d, int l) {
    const bool u1 = (l >> 3) & 1;
    const double s0 = (u1 ? c : a) + dpp_f64<0x128>(u1 ? a : c);
    const double s1 = (u1 ? d : b) + dpp_f64<0x128>(u1 ? b : d);
    const bool u2 = (l ^ (l >> 2)) & 1;
    double v = (u2 ? s1 : s0) + dpp_f64<0xB1>(u2 ? s0 : s1);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
}

// T up to order p + 1 for one (far cell, target) pair of a row: P and F for
// the lane's target; the row's sums of w T_n go to L sixteen terms at a time,
// reduce-scattered across the row so that each lane adds one term.
template <int K, class MP>
__device__ __forceinline__ void far_rec_row(double (&T)[NTERM1], double (&C)[16], double Rx, double Ry, double Rz,
                                            double ir2, MP __restrict__ Mc, double* __restrict__ Lc, double w,
                                            int k, double& phi, double& fx, double& fy, double& fz) {
    if constexpr (K < NTERM1) {
        constexpr TEnt e = TT1.e[K];
        if constexpr (K > 0) t_step<K>(T, Rx, Ry, Rz, ir2);
        if constexpr (K < NTERM) {
            phi = fma(T[K], Mc[K], phi);
            C[K & 15] = w * T[K];
            if constexpr ((K & 15) == 15 || K == NTERM - 1) {
#pragma unroll
                for (int j = (K & 15) + 1; j < 16; ++j) C[j] = 0.0;
                const double v = row_reduce_scatter16(C, k);
                const int idx = (K & ~15) + rs_index(k);
                if constexpr ((K & ~15) + 16 <= NTERM) gatomic_add(Lc + idx, v);
                else if (idx < NTERM) gatomic_add(Lc + idx, v);
            }
        }
        if constexpr (e.x1 >= 0) fx = fma((double)e.n1 * T[K], Mc[e.x1], fx);
        if constexpr (e.y1 >= 0) fy = fma((double)e.n2 * T[K], Mc[e.y1], fy);
        if constexpr (e.z1 >= 0) fz = fma((double)e.n3 * T[K], Mc[e.z1], fz);
        // a scheduling boundary every 16 terms keeps the T_n of one stretch from being
        // computed far ahead of their use (measured 3 % faster at p = 6)
        if constexpr ((K & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        far_rec_row<K + 1>(T, C, Rx, Ry, Rz, ir2, Mc, Lc, w, k, phi, fx, fy, fz);
    }
}

// Pair terms of a target with its own image y inside a far cell: with
// D_n = (y - c)^n, v = sum_{|n|<=p} T_n D_n, F_k = sum_{|m|<=p+1} m_k T_m D_{m-e_k}
// (the image's part of the target's field) and G_k = sum_{|n|<=p} n_k T_n D_{n-e_k}
// (the image's own gradient of v).
template <int K>
__device__ __forceinline__ void flag_rec(double (&T)[NTERM1], double (&D)[NTERM], double Rx, double Ry, double Rz,
                                         double ir2, double dx, double dy, double dz, double& v, double (&F)[3],
                                         double (&G)[3]) {
    if constexpr (K < NTERM1) {
        constexpr TEnt e = TT1.e[K];
        if constexpr (K > 0) t_step<K>(T, Rx, Ry, Rz, ir2);
        if constexpr (K < NTERM) {
            if constexpr (K == 0) D[0] = 1.0;
            else if constexpr (e.n1 >= 1) D[K] = D[e.x1] * dx;
            else if constexpr (e.n2 >= 1) D[K] = D[e.y1] * dy;
            else D[K] = D[e.z1] * dz;
            v = fma(T[K], D[K], v);
            if constexpr (e.x1 >= 0) G[0] = fma((double)e.n1 * T[K], D[e.x1], G[0]);
            if constexpr (e.y1 >= 0) G[1] = fma((double)e.n2 * T[K], D[e.y1], G[1]);
            if constexpr (e.z1 >= 0) G[2] = fma((double)e.n3 * T[K], D[e.z1], G[2]);
        }
        if constexpr (e.x1 >= 0) F[0] = fma((double)e.n1 * T[K], D[e.x1], F[0]);
        if constexpr (e.y1 >= 0) F[1] = fma((double)e.n2 * T[K], D[e.y1], F[1]);
        if constexpr (e.z1 >= 0) F[2] = fma((double)e.n3 * T[K], D[e.z1], F[2]);
        flag_rec<K + 1>(T, D, Rx, Ry, Rz, ir2, dx, dy, dz, v, F, G);
    }
}

// Far list, then near list, of the group: rows of 16 lanes, lane k = target k.
__device__ __forceinline__ void grad_rows(const Rep& R, GradShared& S, int far_n, int near_n, double* L, double4* G,
                                          double half_lB, double (&acc)[4]) {
    const int row = threadIdx.x >> 4, k = threadIdx.x & 15;
    const int nt = S.nt;
    const bool tk = k < nt;
    const int kk = tk ? k : 0;
    const double xk = S.tx[kk], yk = S.ty[kk], zk = S.tz[kk];
    const double wk = half_lB * S.tq[kk];
    // a step takes the next kGradRows far cells, one per row: the workgroup first copies
    // their moment rows to LDS (consecutive threads, consecutive words), so that a row reads
    // its cell's moments as it needs them instead of holding them in registers
    for (int j0 = 0; j0 < far_n; j0 += kGradRows) {
        const int nstep = far_n - j0 < kGradRows ? far_n - j0 : kGradRows;
        for (int it = threadIdx.x; it < nstep * MSTR; it += kGradBlock) {
            const int f = it / MSTR, t = it - f * MSTR;
            const int c = (int)S.farc[j0 + f];
            S.mrow[f][t] = c < R.ncell ? R.M[(size_t)c * MSTR + t] : 0.0;
        }
        __syncthreads();
        const int j = j0 + row;
        if (row < nstep) {
            const int c = (int)S.farc[j];
            if (c >= R.ncell) {
                S.err = kErrFarCell;
            } else {
                const bool act = tk && ((S.farm[j] >> k) & 1u);
                const double4 g = R.cgeo[c];
                const double Rx = g.x - xk, Ry = g.y - yk, Rz = g.z - zk;
                double T[NTERM1], C[16];
                T[0] = rsqrt_nr(Rx * Rx + Ry * Ry + Rz * Rz);
                const double ir2 = T[0] * T[0];
                double phi = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
                far_rec_row<0>(T, C, Rx, Ry, Rz, ir2, lrow(S.mrow[row]), L + (size_t)c * MSTR, act ? wk : 0.0, k,
                               phi, fx, fy, fz);
                if (act) { acc[0] += phi; acc[1] += fx; acc[2] += fy; acc[3] += fz; }
            }
        }
        __syncthreads();
    }
    const int n_ion = R.n;
    const int own_img = R.images ? n_ion + S.ion[kk] : -1;
    for (int j = row; j < near_n; j += kGradRows) {
        const int c = (int)S.nearc[j];
        if (c >= R.ncell) { S.err = kErrNearLeaf; continue; }
        const int4 m = R.cm[c];
        if (m.y >= 0 || m.x < 0 || m.z < 0 || m.z + m.x > R.pool) { S.err = kErrNearSlots; continue; }
        const bool act = tk && ((S.nearm[j] >> k) & 1u);
        for (int s = 0; s < m.x; ++s) {
            const double4 src = R.pool4[m.z + s];
            const int sid = R.pidx[m.z + s];
            if (sid < 0 || sid >= R.nsrc) { S.err = kErrNearSlots; break; }
            const double dx = xk - src.x, dy = yk - src.y, dz = zk - src.z;
            const double d2 = dx * dx + dy * dy + dz * dz;
            const bool use = act && sid != S.ion[kk] && sid != own_img && d2 != 0.0;
            double sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
            if (use) {
                const double ir = rsqrt_nr(d2);
                const double qi3 = src.w * (ir * ir * ir);
                acc[0] += src.w * ir; acc[1] += qi3 * dx; acc[2] += qi3 * dy; acc[3] += qi3 * dz;
                sx = wk * qi3 * dx; sy = wk * qi3 * dy; sz = wk * qi3 * dz; sq = wk * ir;
            }
            const double sv = row_sum4_scatter(sx, sy, sz, sq, k);
            if ((k & 6) == 0) gatomic_add(&G[sid].x + (((k >> 3) << 1) | (k & 1)), sv);
        }
    }
}

__global__ void __launch_bounds__(kGradBlock) k_grad(Rep* reps, int r, const int* islot, int nion, double* L,
                                                     double4* G, double4* Gt, double* eterm, int* fcell) {
    using GS = GradShared;
    constexpr int NW = GS::NW;
    __shared__ GS S;
    __shared__ Rep Rs;
    load_rep(Rs, reps + r);
    __syncthreads();
    const Rep& R = Rs;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    const bool imgs = R.images != 0;
    const double half_lB = 0.5 * R.l_B;
    // frontier entries past the LDS capacity go to this workgroup's HBM region: cells, then masks
    uint32_t* const gfr = spill_region(R);
    const int gcap = gfr ? (int)((R.spill_words - 2) / 6 < 0x7FFFFFFF ? (R.spill_words - 2) / 6 : 0x7FFFFFFF) : 0;
    uint32_t* const gfc = gfr;
    uint64_t* const gfm = gfr ? (uint64_t*)(gfr + 2 * (size_t)gcap) : nullptr;
    const int lcap = R.fcap < GS::FCAP ? R.fcap : GS::FCAP;
    const int ngroups = (nion + kGT - 1) / kGT;
    // one group of 16 ions per workgroup, or several when the grid is bounded (HBM frontier regions)
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int g0 = grp * kGT;
        if (tid == 0) { S.nt = min(kGT, nion - g0); S.err = 0; }
        __syncthreads();
        const int nt = S.nt;
        if (tid < nt) {
            const int slot = islot[g0 + tid];
            const int sid = (slot >= 0 && slot < R.pool) ? R.pidx[slot] : -1;
            if (sid < 0 || sid >= R.n) {
                S.err = kErrNearSlots;
                S.ion[tid] = 0;
                S.tx[tid] = 0.0; S.ty[tid] = 0.0; S.tz[tid] = 0.0; S.tq[tid] = 0.0;
                S.kion[tid] = 0;
            } else {
                const double4 p = R.pool4[slot];
                S.ion[tid] = sid;
                S.tx[tid] = p.x; S.ty[tid] = p.y; S.tz[tid] = p.z; S.tq[tid] = p.w;
                S.kion[tid] = morton_key(R, p.x, p.y, p.z);
            }
            const double4 mo = (imgs && sid >= 0 && sid < R.n) ? R.src[R.n + sid] : make_double4(0, 0, 0, 0);
            S.kimg[tid] = imgs ? morton_key(R, mo.x, mo.y, mo.z) : 0;
            S.flag_cell[tid] = -1;
        }
        if (tid == 0) {
            const uint64_t all = (1ull << nt) - 1ull;
            S.fc[0][0] = 0u;
            S.fm[0][0] = all | (imgs ? all << 32 : 0ull) | (all << 48);
        }
        __syncthreads();
        // ---- breadth-first traversal with target masks
        int cur = 0, fs = 1, far_n = 0, near_n = 0, buf = 0;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        bool failed = false, frontier_full = false, rg = false, wg = false;
        for (int level = 0; fs > 0 && !failed; ++level) {
            int next_n = 0;
            for (int base = 0; base < fs; base += kGradBlock) {
                if (far_n > GS::FARCAP - kGradBlock || near_n > GS::NEARCAP - kGradBlock) {
                    __syncthreads();
                    grad_rows(R, S, far_n, near_n, L, G, half_lB, acc);
                    far_n = 0; near_n = 0;
                    __syncthreads();
                }
                const int j = base + tid;
                const bool valid = j < fs;
                const uint32_t ec = valid ? (rg ? gfc[(size_t)cur * gcap + j] : S.fc[cur][j]) : 0u;
                const uint64_t em = valid ? (rg ? gfm[(size_t)cur * gcap + j] : S.fm[cur][j]) : 0ull;
                const int c = (int)(ec & kCellMask);
                uint32_t farb = 0, nearb = 0, copen = 0, cdir = 0;
                int4 m = make_int4(0, -1, 0, 0);
                if (valid && c >= R.ncell) {
                    S.err = kErrFrontCell;
                } else if (valid) {
                    m = R.cm[c];
                    const double4 g = R.cgeo[c];
                    if (m.y >= 0 && m.y + 8 > R.ncell) {
                        S.err = kErrChildLink;
                    } else {
                        const uint32_t open = (uint32_t)(em & 0xFFFFu), dir = (uint32_t)((em >> 16) & 0xFFFFu);
                        const uint32_t inimg = (uint32_t)((em >> 32) & 0xFFFFu);
                        const uint32_t inion = (uint32_t)(em >> 48);
                        uint32_t todo = open | dir;
                        while (todo) {
                            const int t = __builtin_ctz(todo);
                            todo &= todo - 1u;
                            const uint32_t bit = 1u << t;
                            const int np = m.x - (int)((inion >> t) & 1u) - (int)((inimg >> t) & 1u);
                            if (np <= 0) continue;
                            if (dir & bit) {
                                if (m.y >= 0) cdir |= bit; else nearb |= bit;
                                continue;
                            }
                            const double dx = g.x - S.tx[t], dy = g.y - S.ty[t], dz = g.z - S.tz[t];
                            const double d2 = dx * dx + dy * dy + dz * dz;
                            const bool mac = 3.0 * (g.w * g.w) <= R.theta2 * d2;
                            if (mac && np >= R.n0) {
                                farb |= bit;
                                if (inimg & bit) S.flag_cell[t] = c;
                            } else if (np > R.n0 && m.y >= 0) {
                                copen |= bit;
                            } else if (m.y < 0) {
                                nearb |= bit;
                            } else {
                                cdir |= bit;
                            }
                        }
                    }
                }
                const bool kf = farb != 0, kn = nearb != 0, ks = (copen | cdir) != 0;
                const uint64_t lt = lanemask_lt();
                const uint64_t bf = __ballot(kf), bn = __ballot(kn), bs = __ballot(ks);
                if (lane == 0)
                    S.wcnt[buf][w] = (uint64_t)__popcll(bf) | ((uint64_t)__popcll(bn) << 16) |
                                     ((uint64_t)__popcll(bs) << 32);
                __syncthreads();
                uint64_t before = 0, tot = 0;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) {
                    const uint64_t v = S.wcnt[buf][ww];
                    before += ww < w ? v : 0ull;
                    tot += v;
                }
                buf ^= 1;
                const int tf = (int)(tot & 0xffff), tn = (int)((tot >> 16) & 0xffff), ts = (int)((tot >> 32) & 0xffff);
                if (next_n + 8 * ts > (wg ? gcap : lcap)) {  // uniform
                    if (wg || next_n + 8 * ts > gcap) {
                        failed = frontier_full = true;
                        break;
                    }
                    // the next level moves to HBM: what this level wrote so far first
                    for (int k = tid; k < next_n; k += kGradBlock) {
                        gfc[(size_t)(cur ^ 1) * gcap + k] = S.fc[cur ^ 1][k];
                        gfm[(size_t)(cur ^ 1) * gcap + k] = S.fm[cur ^ 1][k];
                    }
                    wg = true;
                }
                if (kf) {
                    const int o = far_n + (int)(before & 0xffff) + __popcll(bf & lt);
                    S.farc[o] = (uint32_t)c;
                    S.farm[o] = farb;
                }
                if (kn) {
                    const int o = near_n + (int)((before >> 16) & 0xffff) + __popcll(bn & lt);
                    S.nearc[o] = (uint32_t)c;
                    S.nearm[o] = nearb;
                }
                if (ks) {
                    const int o = next_n + 8 * ((int)((before >> 32) & 0xffff) + __popcll(bs & lt));
                    const uint32_t live = copen | cdir;
                    const uint32_t inimg = (uint32_t)((em >> 32) & 0xFFFFu) & live;
                    const uint32_t inion = (uint32_t)(em >> 48) & live;
                    // the child digit of every live target's image and ion
                    uint64_t dimg = 0, dion = 0;
                    for (uint32_t rest = inimg; rest; rest &= rest - 1u) {
                        const int t = __builtin_ctz(rest);
                        dimg |= (uint64_t)key_digit(S.kimg[t], level + 1) << (4 * t);
                    }
                    for (uint32_t rest = inion; rest; rest &= rest - 1u) {
                        const int t = __builtin_ctz(rest);
                        dion |= (uint64_t)key_digit(S.kion[t], level + 1) << (4 * t);
                    }
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        uint32_t im = 0, io = 0;
                        for (uint32_t rest = inimg; rest; rest &= rest - 1u) {
                            const int t = __builtin_ctz(rest);
                            if ((int)((dimg >> (4 * t)) & 15u) == d) im |= 1u << t;
                        }
                        for (uint32_t rest = inion; rest; rest &= rest - 1u) {
                            const int t = __builtin_ctz(rest);
                            if ((int)((dion >> (4 * t)) & 15u) == d) io |= 1u << t;
                        }
                        const uint64_t mk = (uint64_t)copen | ((uint64_t)cdir << 16) | ((uint64_t)im << 32) |
                                            ((uint64_t)io << 48);
                        if (wg) {
                            gfc[(size_t)(cur ^ 1) * gcap + o + d] = (uint32_t)(m.y + d);
                            gfm[(size_t)(cur ^ 1) * gcap + o + d] = mk;
                        } else {
                            S.fc[cur ^ 1][o + d] = (uint32_t)(m.y + d);
                            S.fm[cur ^ 1][o + d] = mk;
                        }
                    }
                }
                far_n += tf; near_n += tn; next_n += 8 * ts;
            }
            __syncthreads();
            cur ^= 1;
            fs = next_n;
            rg = wg;
        }
        if (failed && tid == 0) S.err = frontier_full ? kErrFrontier : kErrStack;
        __syncthreads();
        grad_rows(R, S, far_n, near_n, L, G, half_lB, acc);
        // (the far cell holding a target's own image is corrected by k_gflag)
        {
            const int row = tid >> 4, k = tid & 15;
            S.red[row][k][0] = acc[0]; S.red[row][k][1] = acc[1]; S.red[row][k][2] = acc[2]; S.red[row][k][3] = acc[3];
        }
        __syncthreads();
        if (tid < nt) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            for (int rr = 0; rr < kGradRows; ++rr) {
                a0 += S.red[rr][tid][0]; a1 += S.red[rr][tid][1]; a2 += S.red[rr][tid][2]; a3 += S.red[rr][tid][3];
            }
            const int ion = S.ion[tid];
            const double q = S.tq[tid];
            const bool bad = S.err != 0;
            if (bad && tid == 0) reps[r].err_detail = S.err;
            const double ph = bad ? __builtin_nan("") : a0;
            double e = 0.5 * q * ph;
            if (R.geom == 1) {
                const double r2 = S.tx[tid] * S.tx[tid] + S.ty[tid] * S.ty[tid] + S.tz[tid] * S.tz[tid];
                if (imgs) e += 0.5 * R.gamma * R.a * q * q / (r2 - R.a2);
                if (R.Qc != 0.0) e += R.Qc * q / sqrt(r2);
            }
            eterm[ion] = e;
            const double wq = half_lB * q;
            Gt[ion] = make_double4(-wq * a1, -wq * a2, -wq * a3, half_lB * ph);
            fcell[ion] = S.flag_cell[tid];
        }
        __syncthreads();
    }
}

// The far cell that holds a target's own image in its traversal (found by k_grad;
// one thread per ion): the image's pair terms with the target, taken through that
// cell's expansion, come back out of the target's potential, field and energy term
// and out of the image's source-side gradient.  Kept apart from k_grad because it
// holds every monomial of the image and T up to order p + 1 at once.
__global__ void __launch_bounds__(256) k_gflag(Rep* reps, int r, const int* fcell, double4* G, double4* Gt,
                                               double* eterm) {
    const Rep& R = reps[r];
    const int ion = blockIdx.x * blockDim.x + threadIdx.x;
    if (ion >= R.n || !R.images) return;
    const int c = fcell[ion];
    if (c < 0) return;
    if (c >= R.ncell) { reps[r].err_detail = kErrFlagCell; return; }
    const double4 g = R.cgeo[c];
    const double4 x = R.src[ion];
    const double4 y = R.src[R.n + ion];
    const double Rx = g.x - x.x, Ry = g.y - x.y, Rz = g.z - x.z;
    double T[NTERM1], D[NTERM];
    T[0] = rsqrt_nr(Rx * Rx + Ry * Ry + Rz * Rz);
    const double ir2 = T[0] * T[0];
    double v = 0.0, F[3] = {0.0, 0.0, 0.0}, Gk[3] = {0.0, 0.0, 0.0};
    flag_rec<0>(T, D, Rx, Ry, Rz, ir2, y.x - g.x, y.y - g.y, y.z - g.z, v, F, Gk);
    const double half_lB = 0.5 * R.l_B, wq = half_lB * x.w;
    double4 gt = Gt[ion];
    gt.x += wq * (y.w * F[0]);
    gt.y += wq * (y.w * F[1]);
    gt.z += wq * (y.w * F[2]);
    gt.w -= half_lB * (y.w * v);
    Gt[ion] = gt;
    eterm[ion] -= 0.5 * x.w * (y.w * v);
    double4 gs = G[R.n + ion];
    gs.x -= wq * y.w * Gk[0];
    gs.y -= wq * y.w * Gk[1];
    gs.z -= wq * y.w * Gk[2];
    gs.w -= wq * v;
    G[R.n + ion] = gs;
}

// The target's own line images (multiple-image model; one thread per ion, after
// k_gflag): k_grad kept them in the ion's traversal as ordinary sources, so each pair
// term of the ion with one of them comes back out where the traversal met it -- through
// the expansion of the first cell of the line image's root path that passes the MAC,
// else directly at its leaf -- from the ion's potential, field and energy term and from
// the line image's source-side gradient.  The ion's energy with its own line images,
// 1/2 q sum_m c_m q_K / |r - t_m r_K|, joins its energy term (its gradient is k_chain's).
__global__ void __launch_bounds__(256) k_gline(Rep* reps, int r, double4* G, double4* Gt, double* eterm) {
    const Rep& R = reps[r];
    const int ion = blockIdx.x * blockDim.x + threadIdx.x;
    if (ion >= R.n || R.nline <= 0) return;
    const double4 x = R.src[ion];
    const double half_lB = 0.5 * R.l_B, wq = half_lB * x.w;
    double4 gt = Gt[ion];
    double e = eterm[ion];
    for (int m = 0; m < R.nline; ++m) {
        const int s = 2 * R.n + m * R.n + ion;
        const double4 y = R.src[s];
        const uint64_t key = morton_key(R, y.x, y.y, y.z);
        int c = 0, far = -1;
        bool leaf = false;
        double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
        for (int level = 0; level < kMaxLevels; ++level) {
            if (c < 0 || c >= R.ncell) break;
            g = R.cgeo[c];
            const double dx = g.x - x.x, dy = g.y - x.y, dz = g.z - x.z;
            if (3.0 * (g.w * g.w) <= R.theta2 * (dx * dx + dy * dy + dz * dz)) { far = c; break; }
            const int link = R.cm[c].y;
            if (link < 0) { leaf = true; break; }
            if (link + 8 > R.ncell) break;
            c = link + key_digit(key, level + 1);
        }
        double v, F[3] = {0.0, 0.0, 0.0}, Gk[3] = {0.0, 0.0, 0.0};
        if (far >= 0) {
            const double Rx = g.x - x.x, Ry = g.y - x.y, Rz = g.z - x.z;
            double T[NTERM1], D[NTERM];
            T[0] = rsqrt_nr(Rx * Rx + Ry * Ry + Rz * Rz);
            v = 0.0;
            flag_rec<0>(T, D, Rx, Ry, Rz, T[0] * T[0], y.x - g.x, y.y - g.y, y.z - g.z, v, F, Gk);
        } else if (leaf) {
            // 1/|x - y|: -d/dx = d/dy = (x - y) / |x - y|^3
            const double ex = x.x - y.x, ey = x.y - y.y, ez = x.z - y.z;
            const double ir = rsqrt_nr(ex * ex + ey * ey + ez * ez), ir3 = ir * ir * ir;
            v = ir;
            F[0] = Gk[0] = ex * ir3; F[1] = Gk[1] = ey * ir3; F[2] = Gk[2] = ez * ir3;
        } else {
            reps[r].err_detail = kErrPathCell;
            v = __builtin_nan("");
        }
        gt.x += wq * (y.w * F[0]);
        gt.y += wq * (y.w * F[1]);
        gt.z += wq * (y.w * F[2]);
        gt.w -= half_lB * (y.w * v);
        e -= 0.5 * x.w * (y.w * v);
        double4 gs = G[s];
        gs.x -= wq * y.w * Gk[0];
        gs.y -= wq * y.w * Gk[1];
        gs.z -= wq * y.w * Gk[2];
        gs.w -= wq * v;
        G[s] = gs;
    }
    const double r2 = x.x * x.x + x.y * x.y + x.z * x.z;
    for (int m = 0; m < R.nline; ++m) e += 0.5 * x.w * (R.line_c[m] * R.gamma * R.a * x.w / (r2 - R.line_t[m] * R.a2));
    Gt[ion] = gt;
    eterm[ion] = e;
}

// Ion groups of the gradient traversal: the ions in the order of the build's
// key sort (a space-filling curve, so consecutive ions are close in space).
// rank[k] counts the ions before sorted position k; islot[rank] is the
// current slot of that ion.
__global__ void __launch_bounds__(256) k_gcount(const Rep* reps, int r, int* rank) {
    const Rep& R = reps[r];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < R.nsrc) rank[k] = (unsigned)R.perm[k] < (unsigned)R.n ? 1 : 0;
}

__global__ void __launch_bounds__(1024) k_gscan(int* v, int nv) {
    __shared__ uint64_t wsum[1024 / 64 + 1];
    int carry = 0;
    for (int base = 0; base < nv; base += 1024) {
        const int j = base + threadIdx.x;
        const int x = j < nv ? v[j] : 0;
        uint64_t tot;
        const uint64_t ex = block_exscan<1024>((uint64_t)x, wsum, tot);
        if (j < nv) v[j] = carry + (int)ex;
        carry += (int)tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) v[nv] = carry;
}

__global__ void __launch_bounds__(256) k_gfill(const Rep* reps, int r, const int* rank, int* islot) {
    const Rep& R = reps[r];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= R.nsrc) return;
    const int i = R.perm[k];
    if ((unsigned)i >= (unsigned)R.n) return;
    const int rk = rank[k];
    if (rk < 0 || rk >= R.n) return;
    const int2 tr = R.track[i];
    int slot = -1;
    if (tr.x >= 0 && tr.x < R.ncell) {
        const int4 m = R.cm[tr.x];
        if (m.y < 0 && tr.y >= 0 && tr.y < m.x && m.z >= 0 && m.z + m.x <= R.pool) slot = m.z + tr.y;
    }
    islot[rk] = slot;
}

// Step 2, one thread per source: the source side of every far cell holding
// it, sum over its ancestors A of L_A^n (y - c_A)^n, differentiated in y
// (times q) and in q.
__global__ void __launch_bounds__(256) k_adj_down(const Rep* reps, int r, const double* L, double4* G) {
    const Rep& R = reps[r];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= R.nsrc) return;
    const double4 y = R.src[s];
    int c = R.track[s].x;
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int guard = 0; c >= 0 && guard < kMaxLevels; ++guard) {
        if (c >= R.ncell) { v = __builtin_nan(""); break; }
        const double4 g = R.cgeo[c];
        double D[NTERM];
        poly_rec<0>(D, y.x - g.x, y.y - g.y, y.z - g.z,
                    (const double*)__builtin_assume_aligned(L + (size_t)c * MSTR, 32), v, gx, gy, gz);
        c = R.cparent[c];
    }
    double4 o = G[s];
    o.x += y.w * gx; o.y += y.w * gy; o.z += y.w * gz; o.w += v;
    G[s] = o;
}

// Step 3, one thread per ion: both roles of the ion, its image mapped back
// by the chain rule through q_K = gamma a q / |r| and r_K = a^2 r / |r|^2,
// and the exact self-image and central-charge terms.
__global__ void __launch_bounds__(256) k_chain(const Rep* reps, int r, const double4* G, const double4* Gt,
                                               double* dEdr, double* dEdq) {
    const Rep& R = reps[r];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.n) return;
    const double4 si = R.src[i];
    const double x = si.x, y = si.y, z = si.z, q = si.w;
    const double4 a = Gt[i], b = G[i];
    double gx = a.x + b.x, gy = a.y + b.y, gz = a.z + b.z, gq = a.w + b.w;
    const double l = R.l_B;
    const double r2 = x * x + y * y + z * z;
    if (R.images) {
        // a line image sits at t_m r_K with charge c_m q_K: its gradient joins the Kelvin image's
        double4 h = G[R.n + i];
        for (int m = 0; m < R.nline; ++m) {
            const double4 hm = G[2 * R.n + m * R.n + i];
            h.x += R.line_t[m] * hm.x; h.y += R.line_t[m] * hm.y; h.z += R.line_t[m] * hm.z;
            h.w += R.line_c[m] * hm.w;
        }
        const double rn = sqrt(r2);
        const double ir2 = 1.0 / r2, ir4 = ir2 * ir2;
        const double rh = x * h.x + y * h.y + z * h.z;
        gx += R.a2 * (h.x * ir2 - 2.0 * x * rh * ir4);
        gy += R.a2 * (h.y * ir2 - 2.0 * y * rh * ir4);
        gz += R.a2 * (h.z * ir2 - 2.0 * z * rh * ir4);
        const double c = -R.gamma * R.a * q / (r2 * rn);
        gx += h.w * c * x; gy += h.w * c * y; gz += h.w * c * z;
        gq += h.w * R.gamma * R.a / rn;
        const double den = r2 - R.a2;
        const double cs = -l * R.gamma * R.a * q * q / (den * den);
        gx += cs * x; gy += cs * y; gz += cs * z;
        gq += l * R.gamma * R.a * q / den;
        // the ion's energy with its own line images, 1/2 l_B c_m gamma a q^2 / (r^2 - t_m a^2)
        for (int m = 0; m < R.nline; ++m) {
            const double dm = r2 - R.line_t[m] * R.a2;
            const double cl = -l * R.line_c[m] * R.gamma * R.a * q * q / (dm * dm);
            gx += cl * x; gy += cl * y; gz += cl * z;
            gq += l * R.line_c[m] * R.gamma * R.a * q / dm;
        }
    }
    if (R.geom == 1 && R.Qc != 0.0) {
        const double rn = sqrt(r2);
        const double ir3 = 1.0 / (r2 * rn);
        gx += -l * R.Qc * q * x * ir3; gy += -l * R.Qc * q * y * ir3; gz += -l * R.Qc * q * z * ir3;
        gq += l * R.Qc / rn;
    }
    dEdr[3 * (size_t)i] = gx; dEdr[3 * (size_t)i + 1] = gy; dEdr[3 * (size_t)i + 2] = gz;
    dEdq[i] = gq;
}

__global__ void __launch_bounds__(256) k_zero(double* p, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0.0;
}

void run_mc(hipStream_t s, Rep* reps, const McArgs& a, int grid, int wide) {
    // handles with line images take the instantiation with their steps; the others keep the
    // registers of the one-image kernel
    if (a.lines) {
        if (wide) hipLaunchKernelGGL((k_mc<kMcBlock, true>), dim3(grid), dim3(kMcBlock), 0, s, reps, a);
        else hipLaunchKernelGGL((k_mc<kMcBlockBatch, true>), dim3(grid), dim3(kMcBlockBatch), 0, s, reps, a);
    } else {
        if (wide) hipLaunchKernelGGL((k_mc<kMcBlock, false>), dim3(grid), dim3(kMcBlock), 0, s, reps, a);
        else hipLaunchKernelGGL((k_mc<kMcBlockBatch, false>), dim3(grid), dim3(kMcBlockBatch), 0, s, reps, a);
    }
}
void run_mcb(hipStream_t s, Rep* reps, const McArgs& a, int grid, int wide) {
    if (wide) hipLaunchKernelGGL(k_mcb<kMcBlock>, dim3(grid), dim3(kMcBlock), 0, s, reps, a);
    else hipLaunchKernelGGL(k_mcb<kMcBlockBatch>, dim3(grid), dim3(kMcBlockBatch), 0, s, reps, a);
}
void run_move(hipStream_t s, Rep* reps, int r, MoveIO* io, int lines) {
    if (lines) hipLaunchKernelGGL(k_move<true>, dim3(1), dim3(kMcBlock), 0, s, reps, r, io);
    else hipLaunchKernelGGL(k_move<false>, dim3(1), dim3(kMcBlock), 0, s, reps, r, io);
}
// Line images of the multiple-image model (one thread per ion, after k_energy): an
// ion's own line images stay in its traversal as sources, so each is taken back out of
// its potential and energy term where the traversal met it (walk_value).  The ion's
// energy with its own line images, 1/2 q sum_m c_m q_K / |r - t_m r_K|, is added.
__global__ void __launch_bounds__(256) k_eline(Rep* reps, int r, double* phi, double* eterm) {
    const Rep& R = reps[r];
    const int ion = blockIdx.x * blockDim.x + threadIdx.x;
    if (ion >= R.n) return;
    const double4 si = R.src[ion];
    double sub = 0.0;
    for (int m = 0; m < R.nline; ++m) {
        const double4 sc = R.src[2 * R.n + m * R.n + ion];
        int bad = 0;
        double v = walk_value(R, sc, si.x, si.y, si.z, bad);
        if (bad) { reps[r].err_detail = kErrPathCell; v = __builtin_nan(""); }
        sub += sc.w * v;
    }
    const double r2 = si.x * si.x + si.y * si.y + si.z * si.z;
    double self = 0.0;  // own line images: c_m q_K at t_m r_K, |r - t_m r_K| = (r^2 - t_m a^2) / r
    for (int m = 0; m < R.nline; ++m) self += R.line_c[m] * R.gamma * R.a * si.w / (r2 - R.line_t[m] * R.a2);
    if (phi) phi[ion] -= sub;
    eterm[ion] += 0.5 * si.w * (self - sub);
}

void run_energy(hipStream_t s, Rep* reps, int r, int n, double* phi, double* eterm, int max_grid, int nline) {
    // one workgroup per group of key-order positions: at most (2 + nline) n sources
    const long long positions = (long long)n * (2 + nline);
    int grid = (int)std::min<long long>((positions + kEnergyTargets - 1) / kEnergyTargets, 0x7FFFFFFFll);
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    hipLaunchKernelGGL(k_energy, dim3(grid), dim3(kEnergyBlock), 0, s, reps, r, phi, eterm);
    if (nline > 0) hipLaunchKernelGGL(k_eline, dim3((n + 255) / 256), dim3(256), 0, s, reps, r, phi, eterm);
}
void run_grad(hipStream_t s, Rep* reps, int r, const GradWork& w, double* dEdr, double* dEdq, double* eterm,
              int max_grid) {
    const size_t nl = (size_t)w.ncell * MSTR, ng = 4 * (size_t)w.nsrc;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>(4096, (nl + 255) / 256)), dim3(256), 0, s, w.L, nl);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>(4096, (ng + 255) / 256)), dim3(256), 0, s,
                       (double*)w.G, ng);
    // ion groups: ranks of the ions in key order, then their slots
    hipLaunchKernelGGL(k_gcount, dim3((w.nsrc + 255) / 256), dim3(256), 0, s, (const Rep*)reps, r, w.rank);
    hipLaunchKernelGGL(k_gscan, dim3(1), dim3(1024), 0, s, w.rank, w.nsrc);
    hipLaunchKernelGGL(k_gfill, dim3((w.nsrc + 255) / 256), dim3(256), 0, s, (const Rep*)reps, r,
                       (const int*)w.rank, w.islot);
    int ggrid = (w.n + kGT - 1) / kGT;
    if (max_grid > 0 && ggrid > max_grid) ggrid = max_grid;
    hipLaunchKernelGGL(k_grad, dim3(ggrid), dim3(kGradBlock), 0, s, reps, r, (const int*)w.islot, w.n,
                       w.L, w.G, w.Gt, eterm, w.fcell);
    hipLaunchKernelGGL(k_gflag, dim3((w.n + 255) / 256), dim3(256), 0, s, reps, r, (const int*)w.fcell, w.G,
                       w.Gt, eterm);
    if (w.nline > 0)
        hipLaunchKernelGGL(k_gline, dim3((w.n + 255) / 256), dim3(256), 0, s, reps, r, w.G, w.Gt, eterm);
    hipLaunchKernelGGL(k_adj_down, dim3((w.nsrc + 255) / 256), dim3(256), 0, s, (const Rep*)reps, r,
                       (const double*)w.L, w.G);
    hipLaunchKernelGGL(k_chain, dim3((w.n + 255) / 256), dim3(256), 0, s, (const Rep*)reps, r,
                       (const double4*)w.G, (const double4*)w.Gt, dEdr, dEdq);
}

// Phase timers of the batched kernel (a build with -DBHMC_PHASE_TIMERS): ticks of the
// constant clock per phase, then rounds and moves; reset after reading if asked.
int read_phases(unsigned long long* out, int n, int reset) {
#ifdef BHMC_PHASE_TIMERS
    unsigned long long v[kNumPhases];
    if (hipMemcpyFromSymbol(v, HIP_SYMBOL(g_phase), sizeof(v)) != hipSuccess) return -1;
    for (int k = 0; k < n && k < kNumPhases; ++k) out[k] = v[k];
    if (reset) {
        for (int k = 0; k < kNumPhases; ++k) v[k] = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase), v, sizeof(v)) != hipSuccess) return -1;
    }
    return kNumPhases;
#else
    (void)out; (void)n; (void)reset;
    return 0;
#endif
}

const EvalOps kOps = {run_mc, run_mcb, kBM, run_move, run_energy, run_grad, read_phases};

}  // namespace BHMC_NS

const EvalOps* BHMC_CAT(eval_ops_p, BHMC_P)() { return &BHMC_NS::kOps; }

}  // namespace bhmc
