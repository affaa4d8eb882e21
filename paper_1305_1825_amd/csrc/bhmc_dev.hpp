// Device-side data layout and helpers of the bhmc library (gfx950, wave64).
//
// One replica = one octree over its sources (ions 0..n-1, Kelvin images
// n..2n-1).  Every replica owns its own device buffers; the kernels reach them
// through a table of Rep descriptors, so a replica can be rebuilt without
// touching the others.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bhmc {

constexpr int kMaxDepth = 21;
constexpr int kMaxLevels = kMaxDepth + 1;
constexpr int kPMax = 10;

// Device-side index checks: a failed check records one of these codes and the
// access is skipped, so a corrupted index can never reach memory.
enum ErrDetail {
    kErrNone = 0, kErrStack = 1, kErrFrontCell = 2, kErrChildLink = 3, kErrFarCell = 4,
    kErrNearLeaf = 5, kErrNearSlots = 6, kErrOvlLeaf = 7, kErrPathCell = 8, kErrPathDepth = 9,
    kErrCommitLeaf = 10, kErrCommitSlot = 11, kErrCommitSource = 12, kErrFlagCell = 13,
    kErrMomentCell = 14, kErrBuildPerm = 15, kErrBuildCell = 16, kErrBuildPool = 17,
    kErrFrontier = 18  // a level's frontier outgrew its LDS capacity and no HBM region could take it
};

// Per-replica descriptor.  Host writes parameters and pointers, kernels write
// sizes, statuses and the Monte Carlo counters.
struct Rep {
    // ---- parameters (host)
    double lo[3], side, scale;     // root cube and key scale 2^21 / side
    double theta2;                 // theta * theta
    double l_B, a, a2, gamma, Qc;  // Bjerrum length, sphere, gamma, central charge
    double rmin2, rmax2, tau2;     // shell walls (squared), hard core squared
    double reach2;                 // (tau + 1e-12 side)^2: cells within this take the hard-core descent
    double hi[3];                  // lo + side per axis (cube walls)
    int geom, images, leaf_cap, n0, max_depth, slack;
    int far32;                     // far field from the single-precision moments (M32)
    // multiple images: nline line-image points per ion, source 2n + m n + i at line_t[m] times
    // the Kelvin point with line_c[m] times the Kelvin charge (energies only)
    int nline;
    double line_t[8], line_c[8];
    int n, nsrc;
    // ---- sizes (kernels)
    int ncell, nleaf, pool, depth, nsplit;
    int level_start[kMaxLevels + 1];
    int status;                    // build status (0 or a negative bhmc_status)
    // ---- frontier spill (host): a level whose frontier outgrows fcap entries in LDS continues in
    // the HBM region of its workgroup (blockIdx.x < spill_regions), spill_words 32-bit words each
    int fcap;
    int spill_regions;
    long long spill_words;
    uint32_t* spill;
    // ---- buffers
    double4* src;                  // (x, y, z, q) per source, home copy
    uint64_t* keys; int* perm;     // sorted keys and source index, as built
    uint64_t* ktmp; int* ptmp;     // radix-sort ping-pong
    int2* track;                   // tracking of each source: (its leaf's cell, slot)
    double4* cgeo;                 // centre x, y, z and half side h
    int4* cm;                      // (N_A, link, leaf slot base, leaf capacity); link is the
                                   // first child (>= 0) or -1 - leaf; base/cap only for leaves
    int* cparent; int* clevel;
    uint64_t* ckey;                // smallest key of the cell
    int* cbegin; int* cend;        // build range in the sorted order
    double* M;                     // moments, cell-major: M[cell * nterms + k]
    float* M32;                    // single-precision copy read by the far field, or null
    int* lcell; int* lbase; int* lcap;
    double4* pool4;                // (x, y, z, q) in leaf slot order
    int* pidx;                     // source index of each slot
    // ---- Monte Carlo state
    long long move_next, move_end; // next move index, one past the last
    int mc_status;                 // 0, or BHMC_ECAPACITY / BHMC_ESTACK / BHMC_EINTERNAL
    int err_detail;                // which device-side index check failed (0 = none)
    long long stats[6];            // moves, accepted, wall, overlap, metropolis, unused
};

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11: ten rounds of two 32x32->64 multiplications with a Weyl key schedule.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

struct Draw { int i; double dx, dy, dz, alpha; };

// Move m of replica r: ion from w0, displacement from (w2,w3) (w4,w5) (w6,w7),
// Metropolis alpha from (w8,w9).
__device__ __forceinline__ Draw draw_move(uint64_t seed, uint32_t replica, uint64_t m, int n,
                                          double step) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    U4 a = philox10(U4{(uint32_t)m, (uint32_t)(m >> 32), replica, 0u}, k0, k1);
    U4 b = philox10(U4{(uint32_t)m, (uint32_t)(m >> 32), replica, 1u}, k0, k1);
    U4 c = philox10(U4{(uint32_t)m, (uint32_t)(m >> 32), replica, 2u}, k0, k1);
    Draw d;
    d.i = (int)(((uint64_t)a.x * (uint64_t)(uint32_t)n) >> 32);
    d.dx = step * (u53(a.z, a.w) - 0.5);
    d.dy = step * (u53(b.x, b.y) - 0.5);
    d.dz = step * (u53(b.z, b.w) - 0.5);
    d.alpha = u53(c.x, c.y);
    return d;
}

// ------------------------------------------------------------ keys
// k = min(2^21 - 1, floor((v - lo) scale)), clamped in floating point before the
// conversion so that it is defined for every input (a position outside the root
// cube maps to the nearest face cell).
__device__ __forceinline__ uint32_t quantize(double v, double lo, double scale) {
    double f = floor((v - lo) * scale);
    f = f >= 0.0 ? f : 0.0;
    f = f <= 2097151.0 ? f : 2097151.0;
    return (uint32_t)f;
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x | (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x | (x >> 8)) & 0x001F0000FF0000FFull;
    x = (x | (x >> 16)) & 0x001F00000000FFFFull;
    x = (x | (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}

__device__ __forceinline__ uint64_t morton_key(const Rep& R, double x, double y, double z) {
    uint32_t kx = quantize(x, R.lo[0], R.scale);
    uint32_t ky = quantize(y, R.lo[1], R.scale);
    uint32_t kz = quantize(z, R.lo[2], R.scale);
    return (spread3(kx) << 2) | (spread3(ky) << 1) | spread3(kz);
}

// digit of a key at level l >= 1: 4 x + 2 y + z
__device__ __forceinline__ int key_digit(uint64_t key, int level) {
    return (int)((key >> (63 - 3 * level)) & 7u);
}

// ------------------------------------------------------------ geometry
// Kelvin image: charge gamma a q / |r| at (a^2 / |r|^2) r.
__device__ __forceinline__ double4 kelvin(const Rep& R, double x, double y, double z, double q) {
    double r2 = x * x + y * y + z * z;
    double s = R.a2 / r2;
    double rn = sqrt(r2);
    return make_double4(s * x, s * y, s * z, ((R.gamma * R.a) * q) / rn);
}

__device__ __forceinline__ bool outside(const Rep& R, double x, double y, double z) {
    if (R.geom == 0)
        return x < R.lo[0] || x >= R.hi[0] || y < R.lo[1] || y >= R.hi[1] || z < R.lo[2] ||
               z >= R.hi[2];
    double r2 = x * x + y * y + z * z;
    return r2 <= R.rmin2 || r2 >= R.rmax2;
}

__device__ __forceinline__ bool in_root(const Rep& R, double x, double y, double z) {
    return x >= R.lo[0] && x < R.hi[0] && y >= R.lo[1] && y < R.hi[1] && z >= R.lo[2] &&
           z < R.hi[2];
}

// 1/sqrt(x): hardware FP64 estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2, each of which doubles the number of correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// ------------------------------------------------------------ block primitives
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl_up((int)lo, d, 64);
    hi = (uint32_t)__shfl_up((int)hi, d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Exclusive block scan of a uint64 (packed counters add lane-wise as long
// as no field overflows).  wsum: LDS, BLOCK/64 + 1 entries.  The caller must
// place a barrier between two calls that share wsum.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_exscan(uint64_t v, uint64_t* wsum, uint64_t& total) {
    constexpr int NW = BLOCK / 64;
    const int lane = lane_id(), w = wave_id();
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = shfl_up_u64(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) { uint64_t t = wsum[k]; wsum[k] = s; s += t; }
        wsum[NW] = s;
    }
    __syncthreads();
    total = wsum[NW];
    return wsum[w] + x - v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace bhmc
