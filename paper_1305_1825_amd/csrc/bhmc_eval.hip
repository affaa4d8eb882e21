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
struct TTab { TEnt e[NTERM]; };

constexpr TTab make_tab() {
    TTab t{};
    int k = 0;
    for (int s = 0; s <= P; ++s)
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
constexpr TTab TT = make_tab();

struct MiTab { int v[3 * NTERM]; };
constexpr MiTab make_mi() {
    MiTab m{};
    for (int k = 0; k < NTERM; ++k) { m.v[3 * k] = TT.e[k].n1; m.v[3 * k + 1] = TT.e[k].n2; m.v[3 * k + 2] = TT.e[k].n3; }
    return m;
}
__constant__ MiTab c_mi = make_mi();

// d^n by repeated multiplication (x, then y, then z), as the moments are built
__device__ __forceinline__ double mono(int k, double dx, double dy, double dz) {
    const int n1 = c_mi.v[3 * k], n2 = c_mi.v[3 * k + 1], n3 = c_mi.v[3 * k + 2];
    double v = 1.0;
    for (int e = 0; e < n1; ++e) v *= dx;
    for (int e = 0; e < n2; ++e) v *= dy;
    for (int e = 0; e < n3; ++e) v *= dz;
    return v;
}

// ------------------------------------------------------------ far field
// T_n(R) by eq. 3.4 with T_0 = 1/|R|:
//   T_n = -[ (2s-1)/s sum_i R_i T_{n-e_i} + (s-1)/s sum_i T_{n-2e_i} ] / |R|^2,
// accumulated into sum_n T_n M^n as soon as each T_n exists.
template <int K>
__device__ __forceinline__ void far_rec(double (&T)[NTERM], double Rx, double Ry, double Rz,
                                        double ir2, const double* __restrict__ Mc, double& acc) {
    if constexpr (K < NTERM) {
        constexpr TEnt e = TT.e[K];
        if constexpr (K > 0) {
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
        acc = fma(T[K], Mc[K], acc);
        far_rec<K + 1>(T, Rx, Ry, Rz, ir2, Mc, acc);
    }
}

__device__ __forceinline__ double far_eval(double Rx, double Ry, double Rz, const double* Mc) {
    const double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    double T[NTERM];
    T[0] = rsqrt_nr(r2);
    const double ir2 = T[0] * T[0];
    double acc = 0.0;
    far_rec<0>(T, Rx, Ry, Rz, ir2, Mc, acc);
    return acc;
}

// ------------------------------------------------------------ traversal state
constexpr uint32_t kCellMask = 0xFFFFFFu;
constexpr uint32_t kFlagIon = 1u << 28, kFlagImg = 1u << 29, kFlagDirect = 1u << 30;

__device__ __forceinline__ uint32_t pack(int cell, int t, uint32_t flags) {
    return (uint32_t)cell | ((uint32_t)t << 24) | flags;
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
    int near_pre[NEARCAP + 1];
    int near_base[NEARCAP];
    uint32_t flagl[2 * NTG];
    double Mx[2 * NTG][MSTR];
    double tx[NTG], ty[NTG], tz[NTG];
    int ex_i[NTG], ex_k[NTG];
    uint64_t kx_i[NTG], kx_k[NTG];
    double4 es_i[NTG], es_k[NTG];
    uint32_t ovl[OVLCAP];
    int n_ovl, ovl_t, ovl_ex;
    int err, overlap, coincide;
    uint64_t wsum[NW + 1];
    double red[NW][NTG];
    double res[NTG];
};

template <int NTG>
__device__ __forceinline__ void add_to(double (&acc)[NTG], int t, double v) {
#pragma unroll
    for (int k = 0; k < NTG; ++k)
        if (k == t) acc[k] += v;
}

template <int NTG, int BLOCK>
__device__ void flush_far(const Rep& R, Trav<NTG, BLOCK>& S, int far_n, double (&acc)[NTG]) {
    for (int j = threadIdx.x; j < far_n; j += BLOCK) {
        const uint32_t e = S.farl[j];
        const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const double4 g = R.cgeo[c];
        const double* Mc = (const double*)__builtin_assume_aligned(R.M + (size_t)c * MSTR, 32);
        add_to<NTG>(acc, t, far_eval(g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t], Mc));
    }
}

// Near leaves: direct sum over the leaf's index array (slot order).  For the
// overlap target every ion other than the mover within tau is an overlap.
template <int NTG, int BLOCK>
__device__ void flush_near(const Rep& R, Trav<NTG, BLOCK>& S, int near_n, double (&acc)[NTG]) {
    for (int j = threadIdx.x; j < near_n; j += BLOCK) {
        const uint32_t e = S.nearl[j];
        const int c = (int)(e & kCellMask);
        int base = 0, cnt = 0;
        if (c < R.ncell) {
            const int leaf = -1 - R.clink[c];
            if (leaf >= 0 && leaf < R.nleaf) {
                base = R.lbase[leaf];
                cnt = R.ccount[c];
                if (cnt < 0 || cnt > R.lcap[leaf] || base < 0 || base + cnt > R.pool) {
                    S.err = kErrNearSlots;
                    cnt = 0;
                }
            } else {
                S.err = kErrNearLeaf;
            }
        } else {
            S.err = kErrNearLeaf;
        }
        S.near_base[j] = base;
        S.near_pre[j] = cnt;
    }
    __syncthreads();
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
    const int total = carry;
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
    __syncthreads();
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
__device__ void overlap_below_far(const Rep& R, Trav<NTG, BLOCK>& S) {
    __shared__ int s_cnt[2];
    const int t = S.ovl_t;
    const double x = S.tx[t], y = S.ty[t], z = S.tz[t];
    const double reach = sqrt(R.tau2) + 1e-12 * R.side;
    const double reach2 = reach * reach;
    // n_ovl counts every insert attempt; entries past OVLCAP were never stored
    int cur = 0, fs = S.n_ovl < Trav<NTG, BLOCK>::OVLCAP ? S.n_ovl : Trav<NTG, BLOCK>::OVLCAP;
    for (int j = threadIdx.x; j < fs; j += BLOCK) S.front[0][j] = S.ovl[j];
    while (fs > 0) {
        if (threadIdx.x == 0) s_cnt[cur ^ 1] = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < fs; j += BLOCK) {
            const int c = (int)S.front[cur][j];
            if (c < 0 || c >= R.ncell) { S.err = kErrOvlLeaf; continue; }
            const int link = R.clink[c];
            if (link >= 0 && link + 8 > R.ncell) { S.err = kErrChildLink; continue; }
            if (link < 0) {
                const int leaf = -1 - link;
                if (leaf >= R.nleaf) { S.err = kErrOvlLeaf; continue; }
                const int base = R.lbase[leaf], cnt = R.ccount[c];
                if (cnt < 0 || base < 0 || base + cnt > R.pool) { S.err = kErrOvlLeaf; continue; }
                for (int k = 0; k < cnt; ++k) {
                    const int sid = R.pidx[base + k];
                    if (sid >= R.n || sid == S.ovl_ex) continue;
                    const double4 s = R.pool4[base + k];
                    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
                    if (dx * dx + dy * dy + dz * dz <= R.tau2) S.overlap = 1;
                }
            } else {
                for (int d = 0; d < 8; ++d) {
                    const int ch = link + d;
                    if (R.ccount[ch] == 0) continue;
                    if (box_dist2(R.cgeo[ch], x, y, z) <= reach2) {
                        const int slot = atomicAdd(&s_cnt[cur ^ 1], 1);
                        if (slot < Trav<NTG, BLOCK>::FCAP) S.front[cur ^ 1][slot] = (uint32_t)ch;
                        else S.err = kErrStack;
                    }
                }
            }
        }
        __syncthreads();
        fs = s_cnt[cur ^ 1];
        if (fs > Trav<NTG, BLOCK>::FCAP) fs = Trav<NTG, BLOCK>::FCAP;
        cur ^= 1;
        __syncthreads();
    }
}

// Breadth-first MAC traversal from the entries already in front[0].  On
// return S.res[t] holds the potential at target t from every source except
// the target's excluded ones, S.err is set if an LDS list overflowed, and
// S.overlap / S.coincide report hard-core hits at the overlap target.
template <int NTG, int BLOCK, class Hook>
__device__ int traverse(const Rep& R, Trav<NTG, BLOCK>& S, int nroot, Hook&& hook) {
    using TS = Trav<NTG, BLOCK>;
    const int tid = threadIdx.x;
    double acc[NTG];
#pragma unroll
    for (int k = 0; k < NTG; ++k) acc[k] = 0.0;
    int cur = 0, fs = nroot, far_n = 0, near_n = 0, nflag = 0;
    bool failed = false;
    int level = 0;
    for (; fs > 0 && !failed; ++level) {
        hook(level);
        int next_n = 0;
        for (int base = 0; base < fs; base += BLOCK) {
            if (far_n > TS::FARCAP - BLOCK) { flush_far<NTG, BLOCK>(R, S, far_n, acc); far_n = 0; __syncthreads(); }
            if (near_n > TS::NEARCAP - BLOCK) { flush_near<NTG, BLOCK>(R, S, near_n, acc); near_n = 0; }
            const int j = base + tid;
            const bool valid = j < fs;
            const uint32_t e = valid ? S.front[cur][j] : 0u;
            const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
            const int fi = (e & kFlagIon) ? 1 : 0, fk = (e & kFlagImg) ? 1 : 0;
            int kind = 0, link = 0;
            uint32_t cdir = e & kFlagDirect;
            if (valid && c >= R.ncell) {
                S.err = kErrFrontCell;
            } else if (valid) {
                const int np = R.ccount[c] - fi - fk;
                link = R.clink[c];
                if (link >= 0 && link + 8 > R.ncell) {
                    S.err = kErrChildLink;
                } else if (np > 0) {
                    if (cdir) {
                        kind = link >= 0 ? 3 : 2;
                    } else {
                        const double4 g = R.cgeo[c];
                        const double dx = g.x - S.tx[t], dy = g.y - S.ty[t], dz = g.z - S.tz[t];
                        const double d2 = dx * dx + dy * dy + dz * dz;
                        const bool mac = 3.0 * (g.w * g.w) <= R.theta2 * d2;
                        if (mac && np >= R.n0) {
                            kind = (fi | fk) ? 4 : 1;
                            if (t == S.ovl_t) {
                                const double reach = sqrt(R.tau2) + 1e-12 * R.side;
                                if (box_dist2(g, S.tx[t], S.ty[t], S.tz[t]) <= reach * reach) {
                                    const int slot = atomicAdd(&S.n_ovl, 1);
                                    if (slot < TS::OVLCAP) S.ovl[slot] = (uint32_t)c; else S.err = kErrStack;
                                }
                            }
                        } else if (np > R.n0 && link >= 0) {
                            kind = 3;
                        } else if (link < 0) {
                            kind = 2;
                        } else {
                            kind = 3;
                            cdir = kFlagDirect;  // N_A <= N_0: sum every source below directly
                        }
                    }
                }
            }
            const uint64_t v = (uint64_t)(kind == 1) | ((uint64_t)(kind == 2) << 16) |
                               ((uint64_t)(kind == 3) << 32) | ((uint64_t)(kind == 4) << 48);
            uint64_t tot;
            const uint64_t ex = block_exscan<BLOCK>(v, S.wsum, tot);
            const int tf = (int)(tot & 0xffff), tn = (int)((tot >> 16) & 0xffff);
            const int ts = (int)((tot >> 32) & 0xffff), tg = (int)(tot >> 48);
            if (next_n + 8 * ts > TS::FCAP || nflag + tg > 2 * NTG) {  // uniform
                failed = true;
                break;
            }
            if (kind == 1) {
                S.farl[far_n + (int)(ex & 0xffff)] = e;
            } else if (kind == 2) {
                S.nearl[near_n + (int)((ex >> 16) & 0xffff)] = e;
            } else if (kind == 4) {
                S.flagl[nflag + (int)(ex >> 48)] = e;
            } else if (kind == 3) {
                const int o = next_n + 8 * (int)((ex >> 32) & 0xffff);
                const int dig_i = fi ? key_digit(S.kx_i[t], level + 1) : -1;
                const int dig_k = fk ? key_digit(S.kx_k[t], level + 1) : -1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const uint32_t fl = (d == dig_i ? kFlagIon : 0u) | (d == dig_k ? kFlagImg : 0u) | cdir;
                    S.front[cur ^ 1][o + d] = pack(link + d, t, fl);
                }
            }
            far_n += tf; near_n += tn; nflag += tg; next_n += 8 * ts;
            __syncthreads();
        }
        cur ^= 1;
        fs = next_n;
    }
    if (failed) {
        if (tid == 0) S.err = kErrStack;
        __syncthreads();
        return level;
    }
    // far cells that hold an excluded source: corrected moments in LDS
    if (nflag > 0) {
        for (int it = tid; it < nflag * NTERM; it += BLOCK) {
            const int f = it / NTERM, k = it % NTERM;
            const uint32_t e = S.flagl[f];
            const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
            if (c >= R.ncell) { S.err = kErrFlagCell; S.Mx[f][k] = 0.0; continue; }
            const double4 g = R.cgeo[c];
            double m = R.M[(size_t)c * MSTR + k];
            if (e & kFlagIon) { const double4 s = S.es_i[t]; m = m - s.w * mono(k, s.x - g.x, s.y - g.y, s.z - g.z); }
            if (e & kFlagImg) { const double4 s = S.es_k[t]; m = m - s.w * mono(k, s.x - g.x, s.y - g.y, s.z - g.z); }
            S.Mx[f][k] = m;
        }
        __syncthreads();
        for (int f = tid; f < nflag; f += BLOCK) {
            const uint32_t e = S.flagl[f];
            const int c = (int)(e & kCellMask), t = (int)((e >> 24) & 15u);
            if (c >= R.ncell) continue;
            const double4 g = R.cgeo[c];
            add_to<NTG>(acc, t, far_eval(g.x - S.tx[t], g.y - S.ty[t], g.z - S.tz[t], S.Mx[f]));
        }
    }
    flush_far<NTG, BLOCK>(R, S, far_n, acc);
    flush_near<NTG, BLOCK>(R, S, near_n, acc);  // ends with a barrier
    if (S.ovl_t >= 0 && S.n_ovl > 0 && S.err == 0) overlap_below_far<NTG, BLOCK>(R, S);
    const int lane = lane_id(), w = wave_id();
#pragma unroll
    for (int k = 0; k < NTG; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) S.red[w][k] = s;
    }
    __syncthreads();
    if (tid < NTG) {
        double s = 0.0;
        for (int ww = 0; ww < TS::NW; ++ww) s += S.red[ww][tid];
        S.res[tid] = s;
    }
    __syncthreads();
    return level;
}

// ------------------------------------------------------------ one Monte Carlo move
struct McShared {
    int path[4][kMaxLevels];  // root paths: ion old, ion new, image old, image new
    int plen[4];
    uint64_t key[4];
    double4 contrib[4];       // (position, charge) of the four contributions
    int ok;
    int err;                  // index-check failure seen while descending or committing
};

struct MoveOut { double dE; int reason; int accepted; int stop; int detail; };

constexpr double kInf = __builtin_huge_val();

// Local modification of Sec. 3.3 for an accepted move: thread 0 moves the ion
// and then its image between leaf index arrays (delete = last entry fills the
// hole; add = append) and keeps the leaf counts; the other threads repair the
// moments and counts of the cells on the four root paths, applying to each
// cell, in order, the old ion (-), new ion (+), old image (-), new image (+).
template <int BLOCK>
__device__ void commit(const Rep& R, McShared& MS, int i) {
    const int tid = threadIdx.x;
    const int nps = R.images ? 4 : 2;
    if (tid == 0) {
        for (int part = 0; part < nps / 2; ++part) {
            const int s = part == 0 ? i : R.n + i;
            const int co = MS.path[2 * part][MS.plen[2 * part] - 1];
            const int cn = MS.path[2 * part + 1][MS.plen[2 * part + 1] - 1];
            const int lo = -1 - R.clink[co], ln = -1 - R.clink[cn];
            const double4 nv = MS.contrib[2 * part + 1];
            if (lo != ln) {
                const int k = R.slot_of[s];
                const int last = R.ccount[co] - 1;
                const int bo = R.lbase[lo];
                const int moved = R.pidx[bo + last];
                R.pool4[bo + k] = R.pool4[bo + last];
                R.pidx[bo + k] = moved;
                if (moved >= 0 && moved < R.nsrc) R.slot_of[moved] = k;
                else MS.err = kErrCommitSource;
                R.ccount[co] = last;
                const int cnt = R.ccount[cn], bn = R.lbase[ln];
                R.pool4[bn + cnt] = nv;
                R.pidx[bn + cnt] = s;
                R.slot_of[s] = cnt;
                R.leaf_of[s] = ln;
                R.ccount[cn] = cnt + 1;
            } else {
                R.pool4[R.lbase[lo] + R.slot_of[s]] = nv;
            }
            R.src[s] = nv;
        }
    }
    int maxlen = 0;
    for (int j = 0; j < nps; ++j) maxlen = MS.plen[j] > maxlen ? MS.plen[j] : maxlen;
    const int items = nps * maxlen * NTERM;
    for (int it = tid; it < items; it += BLOCK) {
        const int k = it % NTERM, rest = it / NTERM;
        const int l = rest % maxlen, j = rest / maxlen;
        if (l >= MS.plen[j]) continue;
        const int c = MS.path[j][l];
        if (c < 0 || c >= R.ncell) continue;  // descents only store checked cells
        bool owner = true;
        for (int jj = 0; jj < j; ++jj)
            if (l < MS.plen[jj] && MS.path[jj][l] == c) owner = false;
        if (!owner) continue;
        const double4 g = R.cgeo[c];
        double m = R.M[(size_t)c * MSTR + k];
        int dc = 0;
        for (int jj = j; jj < nps; ++jj) {
            if (l >= MS.plen[jj] || MS.path[jj][l] != c) continue;
            const double4 s = MS.contrib[jj];
            const double v = mono(k, s.x - g.x, s.y - g.y, s.z - g.z);
            if (jj & 1) { m = m + s.w * v; ++dc; } else { m = m - s.w * v; --dc; }
        }
        R.M[(size_t)c * MSTR + k] = m;
        if (k == 0 && l < MS.plen[j] - 1 && dc != 0) R.ccount[c] += dc;
    }
    __syncthreads();
}

// mode 0: evaluate; 1: Metropolis with alpha, commit if accepted;
// 2: commit unless rejected by a wall or an overlap.
template <int BLOCK>
__device__ MoveOut one_move(const Rep& R, Trav<2, BLOCK>& S, McShared& MS, int i, double rx,
                            double ry, double rz, double alpha, int mode) {
    const int tid = threadIdx.x;
    MoveOut out{kInf, 0, 0, 0, 0};
    const double4 si = R.src[i];
    if (outside(R, rx, ry, rz)) { out.reason = 1; return out; }
    const bool imgs = R.images != 0;
    const int nps = imgs ? 4 : 2;
    if (tid == 0) {
        const double4 sn = make_double4(rx, ry, rz, si.w);
        const double4 mo = imgs ? R.src[R.n + i] : make_double4(0, 0, 0, 0);
        const double4 mn = imgs ? kelvin(R, rx, ry, rz, si.w) : make_double4(0, 0, 0, 0);
        const uint64_t kio = morton_key(R, si.x, si.y, si.z);
        const uint64_t kmo = imgs ? morton_key(R, mo.x, mo.y, mo.z) : 0;
        S.tx[0] = si.x; S.ty[0] = si.y; S.tz[0] = si.z;
        S.tx[1] = rx; S.ty[1] = ry; S.tz[1] = rz;
        for (int t = 0; t < 2; ++t) {
            S.ex_i[t] = i; S.ex_k[t] = imgs ? R.n + i : -1;
            S.kx_i[t] = kio; S.kx_k[t] = kmo;
            S.es_i[t] = si; S.es_k[t] = mo;
        }
        S.ovl_t = 1; S.ovl_ex = i; S.n_ovl = 0;
        S.err = 0; S.overlap = 0; S.coincide = 0;
        const uint32_t fl = kFlagIon | (imgs ? kFlagImg : 0u);
        S.front[0][0] = pack(0, 0, fl);
        S.front[0][1] = pack(0, 1, fl);
        MS.key[0] = kio;
        MS.key[1] = morton_key(R, rx, ry, rz);
        MS.key[2] = kmo;
        MS.key[3] = imgs ? morton_key(R, mn.x, mn.y, mn.z) : 0;
        MS.contrib[0] = si; MS.contrib[1] = sn; MS.contrib[2] = mo; MS.contrib[3] = mn;
    }
    if (tid < 4) { MS.path[tid][0] = 0; MS.plen[tid] = 0; }
    if (tid == 0) MS.err = 0;
    __syncthreads();
    // one step of a root path: descend by the key's digit, or stop at the leaf
    auto step = [&](int level) {
        const int c = MS.path[tid][level];
        const int link = (c >= 0 && c < R.ncell) ? R.clink[c] : -1;
        if (c < 0 || c >= R.ncell || (link >= 0 && link + 8 > R.ncell)) {
            MS.err = kErrPathCell;
            MS.plen[tid] = level + 1;
            MS.path[tid][level] = 0;
        } else if (link >= 0 && level + 1 < kMaxLevels) {
            MS.path[tid][level + 1] = link + key_digit(MS.key[tid], level + 1);
        } else {
            if (link >= 0) MS.err = kErrPathDepth;
            MS.plen[tid] = level + 1;
        }
    };
    // the four root paths descend one level per traversal level
    auto hook = [&](int level) {
        if (tid < nps && MS.plen[tid] == 0 && level < kMaxLevels) step(level);
    };
    const int levels = traverse<2, BLOCK>(R, S, 2, hook);
    if (S.err) { out.stop = S.err == kErrStack ? -7 : -8; out.detail = S.err; __syncthreads(); return out; }
    // the traversal may stop above a path's leaf (a cell holding only the
    // excluded sources, or the image's path): finish those descents
    if (tid < nps) {
        for (int level = levels; MS.plen[tid] == 0 && level < kMaxLevels; ++level) step(level);
        if (MS.plen[tid] == 0) { MS.err = kErrPathDepth; MS.plen[tid] = 1; MS.path[tid][0] = 0; }
    }
    __syncthreads();
    if (MS.err) { out.stop = -8; out.detail = MS.err; __syncthreads(); return out; }
    const double po = S.res[0], pn = S.res[1];
    if (S.overlap || S.coincide) { out.reason = 2; __syncthreads(); return out; }
    const double q = si.w, l = R.l_B;
    double dE = l * q * (pn - po);
    if (R.geom == 1) {
        const double rn2 = rx * rx + ry * ry + rz * rz;
        const double ro2 = si.x * si.x + si.y * si.y + si.z * si.z;
        if (imgs) dE += 0.5 * l * R.gamma * R.a * q * q * (1.0 / (rn2 - R.a2) - 1.0 / (ro2 - R.a2));
        if (R.Qc != 0.0) dE += l * R.Qc * q * (1.0 / sqrt(rn2) - 1.0 / sqrt(ro2));
    }
    out.dE = dE;
    bool acc = false;
    if (mode == 1) acc = dE <= 0.0 || alpha <= exp(-dE);
    else if (mode == 2) acc = true;
    if (!acc) { __syncthreads(); return out; }
    if (tid == 0) {
        // leaves of the four paths and every slot the commit will touch, checked
        bool sane = true;
        int leafc[4] = {0, 0, 0, 0}, leaf[4] = {0, 0, 0, 0};
        for (int j = 0; j < nps; ++j) {
            leafc[j] = MS.path[j][MS.plen[j] - 1];
            const int link = R.clink[leafc[j]];
            leaf[j] = -1 - link;
            if (link >= 0 || leaf[j] >= R.nleaf) sane = false;
        }
        for (int part = 0; sane && part < nps / 2; ++part) {
            const int s = part == 0 ? i : R.n + i;
            if (s < 0 || s >= R.nsrc) { sane = false; break; }
            const int lo = leaf[2 * part];
            const int k = R.slot_of[s], cnt = R.ccount[leafc[2 * part]];
            if (R.leaf_of[s] != lo || k < 0 || k >= cnt || cnt > R.lcap[lo] ||
                R.lbase[lo] + cnt > R.pool || R.pidx[R.lbase[lo] + k] != s)
                sane = false;
        }
        bool ok = sane;
        if (sane) {
            const int lio = leaf[0], lin = leaf[1];
            if (lin != lio && R.ccount[leafc[1]] + 1 > R.lcap[lin]) ok = false;
            if (imgs) {
                const int lmo = leaf[2], lmn = leaf[3];
                if (lmn != lmo) {
                    int c = R.ccount[leafc[3]];
                    if (lin != lio) { if (lmn == lin) c += 1; if (lmn == lio) c -= 1; }
                    if (c + 1 > R.lcap[lmn]) ok = false;
                }
            }
        } else {
            MS.err = kErrCommitSlot;
        }
        MS.ok = ok;
    }
    __syncthreads();
    if (MS.err) { out.stop = -8; out.detail = MS.err; __syncthreads(); return out; }
    if (!MS.ok) { out.stop = -6; __syncthreads(); return out; }
    commit<BLOCK>(R, MS, i);
    out.accepted = 1;
    return out;
}


// ------------------------------------------------------------ kernels
constexpr int kMcBlock = 256;
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
__global__ void __launch_bounds__(kMcBlock) k_mc(Rep* reps, McArgs A) {
    __shared__ Trav<2, kMcBlock> S;
    __shared__ McShared MS;
    __shared__ Rep Rs;
    __shared__ int s_r;
    const int tid = threadIdx.x;
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
        const long long mend = Rs.move_end;
        long long st_moves = 0, st_acc = 0, st_wall = 0, st_ovl = 0, st_met = 0;
        int status = 0, detail = 0;
        for (; m < mend; ++m) {
            const Draw d = draw_move(A.seed, (uint32_t)r, (uint64_t)m, Rs.n, A.step);
            const double4 si = Rs.src[d.i];
            const MoveOut o = one_move<kMcBlock>(Rs, S, MS, d.i, si.x + d.dx, si.y + d.dy,
                                                 si.z + d.dz, d.alpha, 1);
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

__global__ void __launch_bounds__(kMcBlock) k_move(Rep* reps, int r, MoveIO* io) {
    __shared__ Trav<2, kMcBlock> S;
    __shared__ McShared MS;
    __shared__ Rep Rs;
    load_rep(Rs, reps + r);
    __syncthreads();
    const int i = io->i;
    const MoveOut o = one_move<kMcBlock>(Rs, S, MS, i, io->rn[0], io->rn[1], io->rn[2], 0.0,
                                         io->mode == 0 ? 0 : 2);
    if (threadIdx.x == 0) {
        io->dE = o.dE;
        io->reason = o.reason;
        io->status = o.stop;
        if (o.detail) reps[r].err_detail = o.detail;
    }
}

// Potential at every ion (targets in groups of kEnergyTargets per
// workgroup), with the ion and its image excluded, and each ion's term of
//   E / l_B = 1/2 q phi + 1/2 gamma a q^2 / (r^2 - a^2) + Q q / r.
__global__ void __launch_bounds__(kEnergyBlock) k_energy(Rep* reps, int r, double* phi, double* eterm) {
    constexpr int NTG = kEnergyTargets;
    __shared__ Trav<NTG, kEnergyBlock> S;
    __shared__ Rep Rs;
    load_rep(Rs, reps + r);
    __syncthreads();
    const int t0 = blockIdx.x * NTG;
    const int nv = min(NTG, Rs.n - t0);
    const int tid = threadIdx.x;
    const bool imgs = Rs.images != 0;
    if (tid < NTG) {
        const int ion = t0 + tid;
        if (tid < nv) {
            const double4 si = Rs.src[ion];
            const double4 mo = imgs ? Rs.src[Rs.n + ion] : make_double4(0, 0, 0, 0);
            S.tx[tid] = si.x; S.ty[tid] = si.y; S.tz[tid] = si.z;
            S.ex_i[tid] = ion; S.ex_k[tid] = imgs ? Rs.n + ion : -1;
            S.kx_i[tid] = morton_key(Rs, si.x, si.y, si.z);
            S.kx_k[tid] = imgs ? morton_key(Rs, mo.x, mo.y, mo.z) : 0;
            S.es_i[tid] = si; S.es_k[tid] = mo;
            S.front[0][tid] = pack(0, tid, kFlagIon | (imgs ? kFlagImg : 0u));
        }
    }
    if (tid == 0) { S.ovl_t = -1; S.ovl_ex = -1; S.n_ovl = 0; S.err = 0; S.overlap = 0; S.coincide = 0; }
    __syncthreads();
    traverse<NTG, kEnergyBlock>(Rs, S, nv, [](int) {});
    if (tid < nv) {
        const int ion = t0 + tid;
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
}

void run_mc(hipStream_t s, Rep* reps, const McArgs& a, int grid) {
    hipLaunchKernelGGL(k_mc, dim3(grid), dim3(kMcBlock), 0, s, reps, a);
}
void run_move(hipStream_t s, Rep* reps, int r, MoveIO* io) {
    hipLaunchKernelGGL(k_move, dim3(1), dim3(kMcBlock), 0, s, reps, r, io);
}
void run_energy(hipStream_t s, Rep* reps, int r, int n, double* phi, double* eterm) {
    const int grid = (n + kEnergyTargets - 1) / kEnergyTargets;
    hipLaunchKernelGGL(k_energy, dim3(grid), dim3(kEnergyBlock), 0, s, reps, r, phi, eterm);
}

const EvalOps kOps = {run_mc, run_move, run_energy, nullptr, kMcBlock};

}  // namespace BHMC_NS

const EvalOps* BHMC_CAT(eval_ops_p, BHMC_P)() { return &BHMC_NS::kOps; }

}  // namespace bhmc
