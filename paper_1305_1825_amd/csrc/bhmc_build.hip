// Tree construction kernels: one workgroup per replica, or for one large
// replica a grid of workgroups (the _wide, _hist, _scan, _scatter and _fill
// forms, with the same results).
//
//   k_sources   ions copied in, Kelvin (and line) images made, confinement checked, keys
//   k_sort      stable LSD radix sort of (key, source) in LDS-ranked tiles
//   k_count     number of split cells per level, straight from sorted keys
//   k_topology  cells level by level (Sec. 3.2 bisection, adaptive by count)
//   k_leaves    leaf index arrays (pool) and tracking information (Sec. 3.3)
//   k_p2m       leaf moments M^n = sum q (r - c)^n            (eq. 3.3)
//   k_m2m       parent moments from children by the binomial shift, one wave per cell
#include "bhmc_dev.hpp"
#include "bhmc_internal.hpp"

#include <algorithm>

namespace bhmc {

constexpr int kBuildBlock = 1024;

// Ion i of replica R (from the inputs, or from the replica's own ions when x is
// null) with its Kelvin image and line images, keys and identity permutation;
// returns 1 for a non-finite input, 2 for a source outside the shell or root.
__device__ __forceinline__ int make_sources(Rep& R, int i, const double* x, const double* y, const double* z,
                                            const double* q, long long off) {
    const int n = R.n;
    int bad = 0;
    double xi, yi, zi, qi;
    if (x) {
        xi = x[off + i]; yi = y[off + i]; zi = z[off + i]; qi = q[off + i];
    } else {  // rebuild from the replica's own current ions
        double4 s = R.src[i];
        xi = s.x; yi = s.y; zi = s.z; qi = s.w;
    }
    if (!(isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(qi))) bad |= 1;
    else if (outside(R, xi, yi, zi) || !in_root(R, xi, yi, zi)) bad |= 2;
    R.src[i] = make_double4(xi, yi, zi, qi);
    R.keys[i] = morton_key(R, xi, yi, zi);
    R.perm[i] = i;
    if (R.images) {
        double4 im = kelvin(R, xi, yi, zi, qi);
        if (!in_root(R, im.x, im.y, im.z)) bad |= 2;
        R.src[n + i] = im;
        R.keys[n + i] = morton_key(R, im.x, im.y, im.z);
        R.perm[n + i] = n + i;
        // line images (multiple-image model): source 2n + m n + i at t_m r_K, charge c_m q_K
        for (int m = 0; m < R.nline; ++m) {
            const int s = 2 * n + m * n + i;
            const double4 li = make_double4(R.line_t[m] * im.x, R.line_t[m] * im.y, R.line_t[m] * im.z,
                                            R.line_c[m] * im.w);
            R.src[s] = li;
            R.keys[s] = morton_key(R, li.x, li.y, li.z);
            R.perm[s] = s;
        }
    }
    return bad;
}

__device__ __forceinline__ int status_of(int bad) { return (bad & 1) ? -1 : ((bad & 2) ? -2 : 0); }

__global__ void __launch_bounds__(kBuildBlock)
k_sources(Rep* reps, const int* rep_list, const double* x, const double* y, const double* z,
          const double* q, const long long* ion_off) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.x] : blockIdx.x];
    const int n = R.n;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int my_bad = 0;
    const long long off = ion_off ? ion_off[blockIdx.x] : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) my_bad |= make_sources(R, i, x, y, z, q, off);
    if (my_bad) atomicOr(&bad, my_bad);
    __syncthreads();
    if (threadIdx.x == 0) R.status = status_of(bad);
}

// The same for one large replica, one thread per ion over a grid; the checks
// gather in *flag (zero on entry) and k_sources_finish turns them into the
// replica's status and zeroes *flag.
__global__ void __launch_bounds__(256) k_sources_wide(Rep* reps, int r, const double* x, const double* y,
                                                      const double* z, const double* q, const long long* ion_off,
                                                      int* flag) {
    Rep& R = reps[r];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.n) return;
    const int b = make_sources(R, i, x, y, z, q, ion_off ? ion_off[0] : 0);
    if (b) atomicOr(flag, b);
}

__global__ void k_sources_finish(Rep* reps, int r, int* flag) {
    reps[r].status = status_of(*flag);
    *flag = 0;
}

constexpr int kSortNW = kBuildBlock / 64;

// One tile of a stable LSD pass: the items [base, base + kBuildBlock) of (ka, va)
// below n go to (kb, vb) at off[d] plus their rank among the tile's items of
// digit d, and off[] advances by the tile's counts.  An item's rank comes from a
// wave-wide match of its digit (8 ballots) plus the counts of the waves before
// it (wcnt, zero on entry and on return).
__device__ __forceinline__ void sort_tile(const uint64_t* ka, const int* va, uint64_t* kb, int* vb, int base, int n,
                                          int shift, int* off, int (*wcnt)[256], int* tile_tot) {
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    const int k = base + tid;
    const bool valid = k < n;
    const uint64_t key = valid ? ka[k] : 0;
    const int val = valid ? va[k] : 0;
    const int dig = (int)((key >> shift) & 255);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (dig >> b) & 1;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(peers & below);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[w][dig] = __popcll(peers);
    __syncthreads();
    if (tid < 256) {
        int s = 0;
        for (int ww = 0; ww < kSortNW; ++ww) { int c = wcnt[ww][tid]; wcnt[ww][tid] = s; s += c; }
        tile_tot[tid] = s;
    }
    __syncthreads();
    if (valid) {
        const int pos = off[dig] + wcnt[w][dig] + rank;
        kb[pos] = key;
        vb[pos] = val;
    }
    __syncthreads();
    if (tid < 256) {
        off[tid] += tile_tot[tid];
        for (int ww = 0; ww < kSortNW; ++ww) wcnt[ww][tid] = 0;
    }
    __syncthreads();
}

// Stable LSD radix sort, 8 passes of 8 bits, one workgroup per replica.  Each
// pass: LDS histogram, exclusive scan, then the tiles scattered in order.
__global__ void __launch_bounds__(kBuildBlock)
k_sort(Rep* reps, const int* rep_list) {
    constexpr int NW = kSortNW;
    Rep& R = reps[rep_list ? rep_list[blockIdx.x] : blockIdx.x];
    const int n = R.nsrc;
    __shared__ int hist[256];
    __shared__ int wcnt[NW][256];
    __shared__ int tile_tot[256];
    __shared__ int skip;
    uint64_t* ka = R.keys; int* va = R.perm;
    uint64_t* kb = R.ktmp; int* vb = R.ptmp;
    const int tid = threadIdx.x;
    for (int k = tid; k < NW * 256; k += kBuildBlock) (&wcnt[0][0])[k] = 0;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        if (tid < 256) hist[tid] = 0;
        if (tid == 0) skip = 0;
        __syncthreads();
        for (int k = tid; k < n; k += kBuildBlock) atomicAdd(&hist[(ka[k] >> shift) & 255], 1);
        __syncthreads();
        if (tid < 256 && hist[tid] == n) skip = 1;  // every key has this digit: pass is a no-op
        __syncthreads();
        const bool skip_pass = skip;
        __syncthreads();
        if (skip_pass) continue;
        if (tid == 0) {
            int s = 0;
            for (int d = 0; d < 256; ++d) { int c = hist[d]; hist[d] = s; s += c; }
        }
        __syncthreads();
        for (int base = 0; base < n; base += kBuildBlock)
            sort_tile(ka, va, kb, vb, base, n, shift, hist, wcnt, tile_tot);
        uint64_t* tk = ka; ka = kb; kb = tk;
        int* tv = va; va = vb; vb = tv;
    }
    // an odd number of executed passes leaves the result in the temporaries
    if (ka != R.keys) {
        for (int k = tid; k < n; k += kBuildBlock) { R.keys[k] = ka[k]; R.perm[k] = va[k]; }
    }
}

// The same sort for one large replica over a grid of workgroups, three launches
// per pass: block histograms, one scan, block scatters.  Block b takes the tiles
// [b T, (b + 1) T) (T tiles per block); the (digit, block) counts are scanned in
// digit-major order, so each block's items of digit d land after every item of a
// smaller digit and after those of digit d in earlier blocks: the order is the
// one of the sort above.  Every pass runs (a constant digit moves nothing), so
// the result ends in keys / perm after the eighth.
__global__ void __launch_bounds__(kBuildBlock)
k_sort_hist(const Rep* reps, int r, int pass, int tiles_per_block, int* hist) {
    const Rep& R = reps[r];
    const int n = R.nsrc, shift = 8 * pass;
    const uint64_t* ka = (pass & 1) ? R.ktmp : R.keys;
    __shared__ int h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const long long lo = (long long)blockIdx.x * tiles_per_block * kBuildBlock;
    const int hi = (int)std::min<long long>(n, lo + (long long)tiles_per_block * kBuildBlock);
    for (int k = (int)lo + threadIdx.x; k < hi; k += kBuildBlock) atomicAdd(&h[(ka[k] >> shift) & 255], 1);
    __syncthreads();
    if (threadIdx.x < 256) hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of m counts in place, one workgroup, in chunks of 16 counts per
// thread staged through LDS: each chunk is loaded and stored back with coalesced
// accesses, each thread scans its 16 consecutive counts (rows padded by one word
// against bank conflicts), and the thread sums are scanned in LDS (Hillis-Steele)
// on top of the carry of the chunks before.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kScanPer * kBuildBlock;
__device__ __forceinline__ int scan_pad(int i) { return i + i / kScanPer; }

__global__ void __launch_bounds__(kBuildBlock) k_sort_scan(int* v, int m) {
    __shared__ int buf[kScanChunk + kBuildBlock];
    __shared__ int part[2][kBuildBlock];
    __shared__ int carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < m; base += kScanChunk) {  // uniform
        const int len = std::min(kScanChunk, m - base);
        for (int k = tid; k < len; k += kBuildBlock) buf[scan_pad(k)] = v[base + k];
        __syncthreads();
        int c[kScanPer];
        int s = 0;
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = kScanPer * tid + j;
            c[j] = i < len ? buf[scan_pad(i)] : 0;
            s += c[j];
        }
        int cur = 0;
        part[0][tid] = s;
        const int carry0 = carry;
        __syncthreads();
        for (int d = 1; d < kBuildBlock; d <<= 1) {
            part[cur ^ 1][tid] = part[cur][tid] + (tid >= d ? part[cur][tid - d] : 0);
            cur ^= 1;
            __syncthreads();
        }
        int run = carry0 + part[cur][tid] - s;  // exclusive prefix of this thread's counts
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = kScanPer * tid + j;
            if (i < len) buf[scan_pad(i)] = run;
            run += c[j];
        }
        __syncthreads();
        for (int k = tid; k < len; k += kBuildBlock) v[base + k] = buf[scan_pad(k)];
        if (tid == kBuildBlock - 1) carry = run;  // carry0 plus the chunk's total
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBuildBlock)
k_sort_scatter(Rep* reps, int r, int pass, int tiles_per_block, const int* hist) {
    Rep& R = reps[r];
    const int n = R.nsrc, shift = 8 * pass;
    const uint64_t* ka = (pass & 1) ? R.ktmp : R.keys;
    const int* va = (pass & 1) ? R.ptmp : R.perm;
    uint64_t* kb = (pass & 1) ? R.keys : R.ktmp;
    int* vb = (pass & 1) ? R.perm : R.ptmp;
    __shared__ int off[256];
    __shared__ int wcnt[kSortNW][256];
    __shared__ int tile_tot[256];
    for (int k = threadIdx.x; k < kSortNW * 256; k += kBuildBlock) (&wcnt[0][0])[k] = 0;
    if (threadIdx.x < 256) off[threadIdx.x] = hist[threadIdx.x * gridDim.x + blockIdx.x];
    __syncthreads();
    const long long lo = (long long)blockIdx.x * tiles_per_block * kBuildBlock;
    const int hi = (int)std::min<long long>(n, lo + (long long)tiles_per_block * kBuildBlock);
    for (int base = (int)lo; base < hi; base += kBuildBlock) sort_tile(ka, va, kb, vb, base, hi, shift, off, wcnt, tile_tot);
}

// first index in [lo, hi) whose key is >= v
__device__ __forceinline__ int lower_bound_key(const uint64_t* keys, int lo, int hi, uint64_t v) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Cell, leaf and slot counts of a replica with `total` split cells, the deepest
// at level depth - 1.
__device__ __forceinline__ void set_cell_counts(Rep& R, int total, int depth) {
    R.nsplit = total;
    R.ncell = 1 + 8 * total;
    R.nleaf = R.ncell - total;
    R.depth = depth;
    // sum_leaves max(count, cap) <= nsrc + nleaf * leaf_cap; every slot index must fit an int
    const long long pool = (long long)R.slack * ((long long)R.nsrc + (long long)R.nleaf * R.leaf_cap) +
                           (2ll + R.nline) * R.nleaf;
    if (pool > 0x7FFFFFFFll - 64) {
        R.pool = 0;
        R.status = -4;
    } else {
        R.pool = (int)pool;
    }
}

// A cell (level l, prefix P) is split iff it holds more than leaf_cap sources
// and l < max_depth; such a cell's parent holds at least as many, so it was
// split too.  The split cells of level l are therefore the runs of equal
// l-prefix longer than leaf_cap.
__global__ void __launch_bounds__(kBuildBlock)
k_count(Rep* reps, const int* rep_list) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.x] : blockIdx.x];
    const int n = R.nsrc;
    __shared__ int cnt;
    __shared__ int total;
    __shared__ int depth;
    if (threadIdx.x == 0) { total = 0; depth = 0; }
    const uint64_t* keys = R.keys;
    for (int l = 0; l < R.max_depth; ++l) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        const int shift = 63 - 3 * l;
        int mine = 0;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const uint64_t P = keys[k] >> shift;
            if (k > 0 && (keys[k - 1] >> shift) == P) continue;
            const uint64_t next = (P + 1) << shift;  // P < 2^(3l): no overflow
            const int e = (l == 0) ? n : lower_bound_key(keys, k, n, next);
            if (e - k > R.leaf_cap) ++mine;
        }
        if (mine) atomicAdd(&cnt, mine);
        __syncthreads();
        const int c = cnt;
        if (threadIdx.x == 0) { total += c; if (c) depth = l + 1; }
        __syncthreads();
        if (c == 0) break;
    }
    if (threadIdx.x == 0) set_cell_counts(R, total, depth);
}

// The same count for one large replica over a grid: thread k takes key k at
// every level where it starts a run of equal prefix, and stops at the first
// such run that is not split (its runs below are parts of it).  Per-level
// counts go to cnt[] (zero on entry); k_count_finish sums them and zeroes cnt.
__global__ void __launch_bounds__(kBuildBlock) k_count_wide(const Rep* reps, int r, int* cnt) {
    const Rep& R = reps[r];
    const int n = R.nsrc;
    const int k = blockIdx.x * kBuildBlock + threadIdx.x;
    if (k >= n) return;
    const uint64_t* keys = R.keys;
    const uint64_t key = keys[k], prev = k > 0 ? keys[k - 1] : 0;
    for (int l = 0; l < R.max_depth; ++l) {
        const int shift = 63 - 3 * l;
        const uint64_t P = key >> shift;
        if (k > 0 && (prev >> shift) == P) continue;
        const uint64_t next = (P + 1) << shift;
        const int e = (l == 0) ? n : lower_bound_key(keys, k, n, next);
        if (e - k <= R.leaf_cap) break;
        atomicAdd(&cnt[l], 1);
    }
}

__global__ void k_count_finish(Rep* reps, int r, int* cnt) {
    Rep& R = reps[r];
    int total = 0, depth = 0;
    for (int l = 0; l < kCountLevels; ++l) {
        total += cnt[l];
        if (cnt[l]) depth = l + 1;
        cnt[l] = 0;
    }
    set_cell_counts(R, total, depth);
}

__device__ __forceinline__ void cell_geometry(const Rep& R, int level, uint64_t kmin, double4& g) {
    const double h = ldexp(R.side, -(level + 1));
    const int sh = 21 - level;
    const uint32_t ix = compact3(kmin >> 2) >> sh;
    const uint32_t iy = compact3(kmin >> 1) >> sh;
    const uint32_t iz = compact3(kmin) >> sh;
    g.x = R.lo[0] + (double)(2u * ix + 1u) * h;
    g.y = R.lo[1] + (double)(2u * iy + 1u) * h;
    g.z = R.lo[2] + (double)(2u * iz + 1u) * h;
    g.w = h;
}

// Cells in level order; the children of a split cell are consecutive in digit
// order; leaves are numbered in cell order.
__global__ void __launch_bounds__(kBuildBlock)
k_topology(Rep* reps, const int* rep_list) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.x] : blockIdx.x];
    __shared__ uint64_t wsum[kBuildBlock / 64 + 1];
    __shared__ int s_next, s_leaf;
    const int n = R.nsrc;
    const uint64_t* keys = R.keys;
    if (threadIdx.x == 0) {
        R.ckey[0] = 0; R.clevel[0] = 0; R.cparent[0] = -1; R.cbegin[0] = 0; R.cend[0] = n;
        R.cm[0] = make_int4(n, -1, -1, 0);
        double4 g; cell_geometry(R, 0, 0, g); R.cgeo[0] = g;
        R.level_start[0] = 0;
        s_next = 1; s_leaf = 0;
    }
    __syncthreads();
    int ls = 0, le = 1, level = 0;
    while (ls < le) {
        for (int base = ls; base < le; base += kBuildBlock) {
            const int c = base + threadIdx.x;
            const bool valid = c < le;
            int b = 0, e = 0;
            bool split = false;
            if (valid) {
                b = R.cbegin[c]; e = R.cend[c];
                split = (e - b > R.leaf_cap) && level < R.max_depth;
            }
            const uint64_t v = valid ? (split ? 1ull : (1ull << 32)) : 0ull;
            uint64_t tot;
            const uint64_t ex = block_exscan<kBuildBlock>(v, wsum, tot);
            const int next0 = s_next, leaf0 = s_leaf;
            if (valid && split && next0 + 8 * (int)(ex & 0xffffffffu) + 8 > R.ncell) {
                R.status = -5;  // the counting pass and this pass disagree: write nothing
            } else if (valid && split) {
                const int first = next0 + 8 * (int)(ex & 0xffffffffu);
                R.cm[c].y = first;
                const uint64_t pk = R.ckey[c];
                const int csh = 60 - 3 * level;
                int cb = b;
                for (int d = 0; d < 8; ++d) {
                    const uint64_t ck = pk | ((uint64_t)d << csh);
                    const int ce = (d == 7) ? e : lower_bound_key(keys, cb, e, pk | ((uint64_t)(d + 1) << csh));
                    const int ch = first + d;
                    R.ckey[ch] = ck; R.clevel[ch] = level + 1; R.cparent[ch] = c;
                    R.cbegin[ch] = cb; R.cend[ch] = ce;
                    R.cm[ch] = make_int4(ce - cb, -1, -1, 0);
                    double4 g; cell_geometry(R, level + 1, ck, g); R.cgeo[ch] = g;
                    cb = ce;
                }
            } else if (valid && leaf0 + (int)(ex >> 32) >= R.nleaf) {
                R.status = -5;
            } else if (valid) {
                const int leaf = leaf0 + (int)(ex >> 32);
                R.lcell[leaf] = c;
                const int cnt = e - b;
                // + 2 + M: one move inserts at most the ion and its 1 + M images
                const int cap = R.slack * (cnt > R.leaf_cap ? cnt : R.leaf_cap) + 2 + R.nline;
                R.lcap[leaf] = cap;
                R.cm[c] = make_int4(cnt, -1 - leaf, -1, cap);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_next = next0 + 8 * (int)(tot & 0xffffffffu);
                s_leaf = leaf0 + (int)(tot >> 32);
            }
            __syncthreads();
        }
        ++level;
        ls = le;
        le = s_next < R.ncell ? s_next : R.ncell;
        if (threadIdx.x == 0) R.level_start[level] = ls;
    }
    if (threadIdx.x == 0) {
        R.level_start[level] = le;
        for (int l = level + 1; l <= kMaxLevels; ++l) R.level_start[l] = le;
        if (s_next != R.ncell || s_leaf != R.nleaf) R.status = -5;
        R.depth = level - 1;
    }
}

// Members of leaf l in sorted order, with their tracking entries.
__device__ __forceinline__ void fill_leaf(Rep& R, int l) {
    const int c = R.lcell[l];
    if (c < 0 || c >= R.ncell) { R.status = -8; return; }
    const int b = R.cbegin[c], e = R.cend[c], base = R.lbase[l];
    if (b < 0 || e > R.nsrc || b > e || base + (e - b) > R.pool) { R.status = -8; return; }
    R.cm[c].z = base;
    for (int k = b; k < e; ++k) {
        const int s = R.perm[k];
        if (s < 0 || s >= R.nsrc) { R.status = -8; continue; }
        R.pool4[base + k - b] = R.src[s];
        R.pidx[base + k - b] = s;
        R.track[s] = make_int2(c, k - b);
    }
}

// Leaf index arrays: bases by an exclusive scan of the capacities; members
// in sorted order; tracking = (leaf, slot) of every source.  With fill = 0
// only the bases (k_leaves_fill then fills the leaves over a grid).
__global__ void __launch_bounds__(kBuildBlock)
k_leaves(Rep* reps, const int* rep_list, int fill) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.x] : blockIdx.x];
    __shared__ uint64_t wsum[kBuildBlock / 64 + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int nl = R.nleaf;
    for (int base = 0; base < nl; base += kBuildBlock) {
        const int l = base + threadIdx.x;
        const int cap = l < nl ? R.lcap[l] : 0;
        uint64_t tot;
        const uint64_t ex = block_exscan<kBuildBlock>((uint64_t)cap, wsum, tot);
        const int c0 = carry;
        if (l < nl) R.lbase[l] = c0 + (int)ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c0 + (int)tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && carry > R.pool) R.status = -5;
    __syncthreads();
    if (carry > R.pool || R.status || !fill) return;  // uniform: nothing is written past the pool
    for (int l = threadIdx.x; l < nl; l += blockDim.x) fill_leaf(R, l);
}

// The leaves of one replica, one thread per leaf over a grid (after k_leaves with fill = 0;
// a status set by the scan leaves every leaf unwritten).
__global__ void __launch_bounds__(256) k_leaves_fill(Rep* reps, int r) {
    Rep& R = reps[r];
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= R.nleaf || R.status) return;
    fill_leaf(R, l);
}

// multi-index table in graded order, shared by the build kernels
__constant__ int c_mi[kMaxTerms * 3];
__constant__ int c_binom[kPMax + 2][kPMax + 2];

__device__ __forceinline__ int mindex_dev(int n1, int n2, int n3) {
    const int s = n1 + n2 + n3;
    return s * (s + 1) * (s + 2) / 6 + (s - n1) * (s - n1 + 1) / 2 + (s - n1 - n2);
}

// P2M at leaves: one thread per (leaf, term); d^n by repeated multiplication.
// Moments are spread over many workgroups per replica: blockIdx.y picks the
// replica, blockIdx.x a chunk of (cell, term) items.
constexpr int kMomBlock = 256;

__global__ void __launch_bounds__(kMomBlock)
k_p2m(Rep* reps, const int* rep_list, int nterms, int mstride) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.y] : blockIdx.y];
    if (R.status) return;  // a failed build leaves the leaf tables unusable
    const long long items = (long long)R.nleaf * nterms;
    for (long long it = blockIdx.x * (long long)kMomBlock + threadIdx.x; it < items;
         it += (long long)gridDim.x * kMomBlock) {
        const int l = (int)(it / nterms), k = (int)(it % nterms);
        const int c = R.lcell[l];
        if (c < 0 || c >= R.ncell) continue;
        const int n1 = c_mi[3 * k], n2 = c_mi[3 * k + 1], n3 = c_mi[3 * k + 2];
        const double4 g = R.cgeo[c];
        const int base = R.lbase[l], cnt = R.cm[c].x;
        if (cnt < 0 || base < 0 || base + cnt > R.pool) continue;
        double acc = 0.0;
        for (int j = 0; j < cnt; ++j) {
            const double4 s = R.pool4[base + j];
            const double dx = s.x - g.x, dy = s.y - g.y, dz = s.z - g.z;
            double v = 1.0;
            for (int e = 0; e < n1; ++e) v *= dx;
            for (int e = 0; e < n2; ++e) v *= dy;
            for (int e = 0; e < n3; ++e) v *= dz;
            acc += s.w * v;
        }
        R.M[(size_t)c * mstride + k] = acc;
    }
}

// M2M, one wave per split cell of a level (the launches go deepest level
// first).  With child d centred at c + s_d,
// s_d = (+-h/2, +-h/2, +-h/2) (+ on x, y, z where bit 4, 2, 1 of d is set),
//   M^n = sum_d sum_{k <= n} C(n, k) s_d^{n-k} M_d^k,
// and s_d^{n-k} = (h/2)^{|n-k|} times the product of the signs of the axes on
// which n - k is odd.  The wave first combines the eight children of every term
// k into W_k[e] = sum_d (product over the axes set in e of d's sign) M_d^k (an
// 8-point Hadamard transform, in LDS), and then each lane forms its terms n as
//   M^n = sum_{k <= n} C(n, k) (h/2)^{|n-k|} W_k[(n - k) mod 2 per axis]:
// one read per k instead of eight.
constexpr int kM2MWaves = 4;
constexpr int kM2MTerms = (kPMax + 1) * (kPMax + 2) * (kPMax + 3) / 6;

__global__ void __launch_bounds__(64 * kM2MWaves)
k_m2m(Rep* reps, const int* rep_list, int nterms, int mstride, int level) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.y] : blockIdx.y];
    if (R.status || level >= R.depth || nterms > kM2MTerms) return;
    __shared__ double W[kM2MWaves][8][kM2MTerms];
    __shared__ double hpow[kM2MWaves][kPMax + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ls = R.level_start[level], le = R.level_start[level + 1];
    for (int base = ls + blockIdx.x * kM2MWaves; base < le; base += gridDim.x * kM2MWaves) {  // uniform
        const int c = base + w;
        const int first = c < le ? R.cm[c].y : -1;
        const bool split = first >= 0 && first + 8 <= R.ncell;
        if (split) {
            for (int k = lane; k < nterms; k += 64) {
                double m[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) m[d] = R.M[(size_t)(first + d) * mstride + k];
#pragma unroll
                for (int b = 4; b >= 1; b >>= 1)
#pragma unroll
                    for (int d = 0; d < 8; ++d)
                        if (!(d & b)) {
                            const double lo = m[d], hi = m[d | b];
                            m[d] = lo + hi;
                            m[d | b] = hi - lo;
                        }
#pragma unroll
                for (int e = 0; e < 8; ++e) W[w][e][k] = m[e];
            }
            if (lane <= kPMax) {
                const double hc = R.cgeo[c].w * 0.5;
                double v = 1.0;
                for (int e = 0; e < lane; ++e) v *= hc;
                hpow[w][lane] = v;
            }
        }
        __syncthreads();
        if (split) {
            for (int n = lane; n < nterms; n += 64) {
                const int n1 = c_mi[3 * n], n2 = c_mi[3 * n + 1], n3 = c_mi[3 * n + 2];
                double acc = 0.0;
                double b1 = 1.0;  // C(n1, k1)
                for (int k1 = 0; k1 <= n1; ++k1) {
                    double b2 = 1.0;
                    for (int k2 = 0; k2 <= n2; ++k2) {
                        double b3 = 1.0;
                        for (int k3 = 0; k3 <= n3; ++k3) {
                            const int e = (((n1 - k1) & 1) << 2) | (((n2 - k2) & 1) << 1) | ((n3 - k3) & 1);
                            acc += (b1 * b2 * b3) * hpow[w][(n1 - k1) + (n2 - k2) + (n3 - k3)] *
                                   W[w][e][mindex_dev(k1, k2, k3)];
                            b3 = b3 * (double)(n3 - k3) / (double)(k3 + 1);
                        }
                        b2 = b2 * (double)(n2 - k2) / (double)(k2 + 1);
                    }
                    b1 = b1 * (double)(n1 - k1) / (double)(k1 + 1);
                }
                R.M[(size_t)c * mstride + n] = acc;
            }
        }
        __syncthreads();
    }
}

// Single-precision copy of the moments for the far field (replicas built with far32).
__global__ void __launch_bounds__(kMomBlock)
k_m32(Rep* reps, const int* rep_list, int nterms, int mstride) {
    Rep& R = reps[rep_list ? rep_list[blockIdx.y] : blockIdx.y];
    if (R.status || !R.M32) return;
    const long long items = (long long)R.ncell * nterms;
    for (long long it = blockIdx.x * (long long)kMomBlock + threadIdx.x; it < items;
         it += (long long)gridDim.x * kMomBlock) {
        const long long c = it / nterms, k = it % nterms;
        R.M32[c * mstride + k] = (float)R.M[c * mstride + k];
    }
}

// ------------------------------------------------------------ host launchers
hipError_t upload_build_tables(int p, void* pinned) {
    int* mi = (int*)pinned;                        // 3 * kMaxTerms ints
    int (*binom)[kPMax + 2] = (int (*)[kPMax + 2])(mi + 3 * kMaxTerms);
    int k = 0;
    for (int s = 0; s <= p; ++s)
        for (int n1 = s; n1 >= 0; --n1)
            for (int n2 = s - n1; n2 >= 0; --n2) { mi[3 * k] = n1; mi[3 * k + 1] = n2; mi[3 * k + 2] = s - n1 - n2; ++k; }
    for (int a = 0; a <= kPMax + 1; ++a)
        for (int b = 0; b <= kPMax + 1; ++b)
            binom[a][b] = (b == 0) ? 1 : (b > a ? 0 : binom[a - 1][b - 1] + (b <= a - 1 ? binom[a - 1][b] : 0));
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_mi), mi, sizeof(int) * 3 * k);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_binom), binom, sizeof(int) * (kPMax + 2) * (kPMax + 2));
    return e;
}

void launch_sources(hipStream_t s, int nrep, Rep* reps, const int* list, const double* x,
                    const double* y, const double* z, const double* q, const long long* ion_off) {
    hipLaunchKernelGGL(k_sources, dim3(nrep), dim3(kBuildBlock), 0, s, reps, list, x, y, z, q, ion_off);
}
void launch_sort(hipStream_t s, int nrep, Rep* reps, const int* list) {
    hipLaunchKernelGGL(k_sort, dim3(nrep), dim3(kBuildBlock), 0, s, reps, list);
}
void launch_count(hipStream_t s, int nrep, Rep* reps, const int* list) {
    hipLaunchKernelGGL(k_count, dim3(nrep), dim3(kBuildBlock), 0, s, reps, list);
}
void launch_sources_wide(hipStream_t s, Rep* reps, int r, int n, const double* x, const double* y,
                         const double* z, const double* q, const long long* ion_off, int* flag) {
    hipLaunchKernelGGL(k_sources_wide, dim3(std::max(1, (n + 255) / 256)), dim3(256), 0, s, reps, r, x, y, z, q,
                       ion_off, flag);
    hipLaunchKernelGGL(k_sources_finish, dim3(1), dim3(1), 0, s, reps, r, flag);
}
void launch_sort_wide(hipStream_t s, Rep* reps, int r, int nsrc, int* hist) {
    const int tiles = (nsrc + kBuildBlock - 1) / kBuildBlock;
    const int tpb = (tiles + kSortGridMax - 1) / kSortGridMax;
    const int grid = std::max(1, (tiles + tpb - 1) / tpb);
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kBuildBlock), 0, s, reps, r, pass, tpb, hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kBuildBlock), 0, s, hist, 256 * grid);
        hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(kBuildBlock), 0, s, reps, r, pass, tpb, hist);
    }
}
void launch_count_wide(hipStream_t s, Rep* reps, int r, int nsrc, int* cnt) {
    hipLaunchKernelGGL(k_count_wide, dim3(std::max(1, (nsrc + kBuildBlock - 1) / kBuildBlock)), dim3(kBuildBlock), 0, s,
                       reps, r, cnt);
    hipLaunchKernelGGL(k_count_finish, dim3(1), dim3(1), 0, s, reps, r, cnt);
}
void launch_topology(hipStream_t s, int nrep, Rep* reps, const int* list) {
    hipLaunchKernelGGL(k_topology, dim3(nrep), dim3(kBuildBlock), 0, s, reps, list);
}
void launch_leaves(hipStream_t s, int nrep, Rep* reps, const int* list) {
    hipLaunchKernelGGL(k_leaves, dim3(nrep), dim3(kBuildBlock), 0, s, reps, list, 1);
}
void launch_leaves_wide(hipStream_t s, Rep* reps, const int* list, int r, int nleaf) {
    hipLaunchKernelGGL(k_leaves, dim3(1), dim3(kBuildBlock), 0, s, reps, list, 0);
    hipLaunchKernelGGL(k_leaves_fill, dim3(std::max(1, (nleaf + 255) / 256)), dim3(256), 0, s, reps, r);
}
static unsigned chunks(long long items) {
    long long b = (items + kMomBlock - 1) / kMomBlock;
    return (unsigned)std::max(1LL, std::min(b, 8192LL));
}

void launch_moments(hipStream_t s, int nrep, Rep* reps, const int* list, int nterms, int mstride,
                    const Rep* host, const int* host_list) {
    long long leaf_items = 0;
    int depth = 0;
    for (int i = 0; i < nrep; ++i) {
        const Rep& h = host[host_list[i]];
        leaf_items = std::max(leaf_items, (long long)h.nleaf * nterms);
        depth = std::max(depth, h.depth);
    }
    hipLaunchKernelGGL(k_p2m, dim3(chunks(leaf_items), nrep), dim3(kMomBlock), 0, s, reps, list, nterms, mstride);
    for (int level = depth - 1; level >= 0; --level) {
        long long items = 0;
        for (int i = 0; i < nrep; ++i) {
            const Rep& h = host[host_list[i]];
            if (level < h.depth)
                items = std::max(items, (long long)(h.level_start[level + 1] - h.level_start[level]) * nterms);
        }
        const long long cells = items / nterms;
        const unsigned blocks = (unsigned)std::max(1LL, std::min((cells + kM2MWaves - 1) / kM2MWaves, 8192LL));
        hipLaunchKernelGGL(k_m2m, dim3(blocks, nrep), dim3(64 * kM2MWaves), 0, s, reps, list, nterms, mstride, level);
    }
    long long cell_items = 0;
    bool any32 = false;
    for (int i = 0; i < nrep; ++i) {
        const Rep& h = host[host_list[i]];
        cell_items = std::max(cell_items, (long long)h.ncell * nterms);
        any32 = any32 || h.far32;
    }
    if (any32)
        hipLaunchKernelGGL(k_m32, dim3(chunks(cell_items), nrep), dim3(kMomBlock), 0, s, reps, list, nterms, mstride);
}

}  // namespace bhmc
