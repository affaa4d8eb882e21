// Trial moves of one chain evaluated several at a time, with the chain unchanged.
// Included by bhmc_eval.hip inside its per-order namespace (P, NTERM, MSTR and the
// traversal helpers above are in scope).
//
// A round takes the next nb <= kBM trial moves of a chain that move distinct ions
// and evaluates every one of them against the tree as it stands at the start of
// the round: one breadth-first MAC traversal (Sec. 3.2) whose frontier entries
// carry the move they belong to, so the level latency of the traversal is paid
// once per round.  The moves are then decided in order.  An accepted earlier move
// j of the round changed the tree only through its four contributions (old and
// new ion, old and new image).  With N_0 = 0 every decision of the traversal
// depends only on the geometry and on whether a cell holds a source, so the
// potential at a target of a later move b on the tree after j differs from the
// one at the start of the round by exactly those contributions, each taken where
// b's traversal meets the contribution's root path: through the expansion of eq.
// 3.3 at the first cell of the path that passes the MAC, or directly at its leaf.
// The expansion of one point source needs no moments: its order-s block is
// P_s(cos psi) |d|^s / |R|^(s+1) (the Legendre form of the coefficients of eq.
// 3.4).  Hard cores (eq. 2.1) are tested against the start-of-round positions,
// naming the ions of earlier moves of the round, so that an overlap with an ion
// that has moved away no longer counts, and against the new positions of the
// accepted earlier moves.  The accepted moves are then committed in order (Sec.
// 3.3): leaf index arrays by one thread, the moments of every distinct cell of
// their root paths with the contributions applied in move order.  Every result is
// the one the move-by-move chain gives, up to the rounding of the sums.

constexpr int kBM = P <= 8 ? 8 : 2;  // trial moves per round (LDS: p = 8 with 8 moves just fits 160 KB)
constexpr int kBT = 2 * kBM;                         // targets per round: 2b old, 2b + 1 new position
// frontier / list entry: cell (bits 0-23), move (24-26), mask of the move's two targets (27-28),
// the cell holds the move's own ion (29) or image (30)
constexpr int kMvSh = 24;
constexpr int kOpSh = 27;
constexpr uint32_t kMbIon = 1u << 29, kMbImg = 1u << 30;
constexpr int kPathCells = kBM * 4 * kMaxLevels;
constexpr int kChunk = 2;  // frontier entries per lane per chunk of the traversal's level loop

static_assert(kBM <= 8, "the move index has three bits");

// Phase timers of a round (built with -DBHMC_PHASE_TIMERS only): thread 0 adds the
// constant-clock ticks of each phase, and the level loop its counts, to the workgroup's
// accumulators in LDS (no device atomics on the round's path); a workgroup adds them to
// the device array read by bhmc_phase_ticks when it finishes a replica.
enum { kPhSetup = 0, kPhLevels, kPhFlagged, kPhFar, kPhNear, kPhOverlap, kPhPaths, kPhCorr, kPhDecide,
       kPhSlots, kPhMoments, kPhRounds, kPhMoves,
       // counts: level-loop chunks, frontier entries, entries holding no remaining source, far and near list entries
       kPhChunks, kPhEntries, kPhEmpty, kPhFarN, kPhNearN,
       // ticks inside the traversal (overlapping the level loop): path descents, commit prefetch
       kPhHookPath, kPhHookPf, kNumPhases };
#ifdef BHMC_PHASE_TIMERS
__device__ unsigned long long g_phase[kNumPhases];
__shared__ unsigned long long s_phase[kNumPhases];
#define PHASE_START() long long ph_t0_ = wall_clock64()
#define PHASE(k)                                                         \
    do {                                                                 \
        if (threadIdx.x == 0) {                                          \
            const long long ph_t1_ = wall_clock64();                     \
            s_phase[k] += (unsigned long long)(ph_t1_ - ph_t0_);         \
            ph_t0_ = ph_t1_;                                             \
        }                                                                \
    } while (0)
#define PHASE_COUNT(k, v) do { if (threadIdx.x == 0) s_phase[k] += (unsigned long long)(v); } while (0)
#else
#define PHASE_START() do {} while (0)
#define PHASE(k) do {} while (0)
#define PHASE_COUNT(k, v) do {} while (0)
#endif

template <int BLOCK>
struct BTrav {
    static constexpr int FCAP = 4096;
    static constexpr int FARCAP = 2048 + kChunk * BLOCK;
    static constexpr int NEARCAP = 1024 + kChunk * BLOCK;
    static constexpr int OVLCAP = 512;
    static constexpr int NW = BLOCK / 64;
    // the traversal's lists, free once it has ended: then per-axis power tables of the commit
    static constexpr int LISTWORDS = 2 * FCAP + FARCAP + 3 * NEARCAP + 1;
    static constexpr int PWROWS = (LISTWORDS / 2) / (3 * (P + 1));
    union {
        struct {
            uint32_t front[2][FCAP];
            uint32_t farl[FARCAP];
            uint32_t nearl[NEARCAP];
            int near_base[NEARCAP];
            int near_pre[NEARCAP + 1];
        };
        double pw[PWROWS][3][P + 1];  // (x - c_x)^e, (y - c_y)^e, (z - c_z)^e of a path entry
    };
    uint32_t flagl[4 * kBM];
    double Mx[4 * kBM][MSTR];
    uint32_t ovl[OVLCAP];
    int n_ovl, near_tot, err;
    uint64_t wcnt[2][kChunk][NW];
    double red[NW][kBT];
    uint32_t mi[NTERM];
    int cnt2[2];
};

struct BMoves {
    int nb;                        // moves of this round
    int ion[kBM];
    double4 ct[kBM][4];            // contributions: old ion, new ion, old image, new image (position, charge)
    uint64_t key[kBM][4];
    double alpha[kBM];
    int wall[kBM];
    double tx[kBT], ty[kBT], tz[kBT];
    int ovl_fixed[kBM];            // overlaps an ion that stays where it is during the round
    uint32_t ovl_moved[kBM];       // bit j: overlaps the ion of earlier move j at its old position
    double pot[kBT];               // potentials on the tree at the start of the round
    double corr[kBM][kBM][2];      // corr[j][b][t]: what committing move j adds to target (b, t)
    int path[kBM][4][kMaxLevels];  // root paths of the four contributions
    double4 path_geo[kBM][4][kMaxLevels];
    int plen[kBM][4];
    int fs0, level0;
    // commit state of each move's ion (0) and image (1) at the start of the round
    int2 tr[kBM][2];
    int4 lm_old[kBM][2];
    int4 lm_new[kBM][2];
    int last_pidx[kBM][2];
    double4 last_pool[kBM][2];
    int self_pidx[kBM][2];
    int pf_stage[kBM][2];
    // decisions
    int acc[kBM];
    int reason[kBM];
    int ndone;                     // moves decided this round (the round ends there)
    int stop;                      // 0, or -6: the move after the decided ones would overflow a leaf
    int err;
    double dE[kBM];
    // distinct cells of the accepted moves' root paths
    int nlist;
    int pw_rows;
    int list_cell[kPathCells];
    uint32_t list_mask[kPathCells];  // bit 4 j + cc: contribution cc of move j applies
    int list_at[kPathCells];         // (j * 4 + cc) * kMaxLevels + level of its geometry; bit 30: internal
    // per pair (b, j < b): b's new position overlaps j's new one (bit j), and how committing j
    // changes the counts of b's new ion leaf and new image leaf; per move: the energy change
    // terms outside the traversal and whether its tracked leaves are where its keys lead
    uint32_t ovl_new[kBM];
    int e_ion[kBM][kBM], e_img[kBM][kBM];
    double dE0[kBM];
    int sane[kBM];
    // leaf index array operations of the accepted moves: lane 4b + k, k = ion old, ion new,
    // image old, image new; type 0 none, 1 delete, 2 append, 3 new position in place
    int op_type[4 * kBM], op_cell[4 * kBM], op_src[4 * kBM], op_slot[4 * kBM];
    int op_base[4 * kBM], op_count[4 * kBM];
    int pw_row[4 * kBM];  // first power-table row of the root path of contribution (j, cc), or -1
    // trial moves drawn ahead, one per lane of the first wave
    int dr_i[kDrawBatch];
    double dr_d[kDrawBatch][4];
};

__device__ __forceinline__ int mv_of(uint32_t e) { return (int)((e >> kMvSh) & 7u); }

template <int NT>
__device__ __forceinline__ void add_to_t(double (&acc)[NT], int t, double v) {
#pragma unroll
    for (int k = 0; k < NT; ++k)
        if (k == t) acc[k] += v;
}

// Sum over the lanes of a wave with the same parity as this one: a lane of parity tb
// accumulates target tb of every move (see far_pass_mb), so lanes 0 and 1 end with the
// wave's sums for the old and the new positions.
__device__ __forceinline__ double wave_sum_parity(double v) {
#pragma unroll
    for (int off = 32; off >= 2; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// An overlap of move b's new position with source sid (an ion other than the mover,
// or any source at distance zero), recorded by name when the ion belongs to an
// earlier move of the round.
__device__ __forceinline__ void record_overlap(BMoves& MV, int b, int sid, int n_ion) {
    uint32_t mv = 0;
    if (sid >= 0 && sid < n_ion)
        for (int j = 0; j < b; ++j)
            if (MV.ion[j] == sid) mv |= 1u << j;
    if (mv) atomicOr(&MV.ovl_moved[b], mv);
    else atomicOr(&MV.ovl_fixed[b], 1);
}

// Exclusive scan of the near leaves' slot counts (as near_scan).
template <int BLOCK>
__device__ int near_scan_mb(BTrav<BLOCK>& S, int near_n) {
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
    __shared__ uint64_t wsum[BLOCK / 64 + 1];
    int carry = 0;
    for (int base = 0; base < near_n; base += BLOCK) {
        const int j = base + threadIdx.x;
        const int v = j < near_n ? S.near_pre[j] : 0;
        uint64_t tot;
        const uint64_t ex = block_exscan<BLOCK>((uint64_t)v, wsum, tot);
        if (j < near_n) S.near_pre[j] = carry + (int)ex;
        carry += (int)tot;
        __syncthreads();
    }
    return carry;
}

// Far cells by lane pairs: the lane of parity tb evaluates target tb (old or new
// position) of the entry's move, both lanes reading the same moment row; acc[b] of a
// lane holds its target of move b.
template <int BLOCK>
__device__ __forceinline__ void far_pass_mb(const Rep& R, BTrav<BLOCK>& S, const BMoves& MV, int far_n, int nflag,
                                            double (&acc)[kBM]) {
    const int tb = (int)(threadIdx.x & 1);
    for (int j2 = threadIdx.x; j2 < 2 * far_n; j2 += BLOCK) {
        const uint32_t e = S.farl[j2 >> 1];
        if (!((e >> (kOpSh + tb)) & 1u)) continue;
        const int c = (int)(e & kCellMask);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const int b = mv_of(e), t = 2 * b + tb;
        const double4 g = gload(R.cgeo + c);
        add_to_t<kBM>(acc, b, far_value(R, c, g.x - MV.tx[t], g.y - MV.ty[t], g.z - MV.tz[t]));
    }
    for (int j2 = threadIdx.x; j2 < 2 * nflag; j2 += BLOCK) {
        const uint32_t e = S.flagl[j2 >> 1];
        if (!((e >> (kOpSh + tb)) & 1u)) continue;
        const int c = (int)(e & kCellMask);
        if (c >= R.ncell) { S.err = kErrFarCell; continue; }
        const int b = mv_of(e), t = 2 * b + tb;
        const double4 g = gload(R.cgeo + c);
        add_to_t<kBM>(acc, b, far_eval(g.x - MV.tx[t], g.y - MV.ty[t], g.z - MV.tz[t], lrow(S.Mx[j2 >> 1])));
    }
}

// Near leaves by lane pairs as the far cells: slot f of the flattened near leaves is
// taken by lanes 2f (old position) and 2f + 1 (new position); for the new position,
// every ion other than the mover within tau is an overlap.
template <int BLOCK>
__device__ __forceinline__ void near_pass_mb(const Rep& R, BTrav<BLOCK>& S, BMoves& MV, int near_n, int total,
                                             double (&acc)[kBM]) {
    const int n_ion = R.n;
    const int tb = (int)(threadIdx.x & 1);
    for (int f2 = threadIdx.x; f2 < 2 * total; f2 += BLOCK) {
        const int f = f2 >> 1;
        int lo = 0, hi = near_n - 1;  // last j with near_pre[j] <= f
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.near_pre[mid] <= f) lo = mid; else hi = mid - 1;
        }
        const uint32_t e = S.nearl[lo];
        if (!((e >> (kOpSh + tb)) & 1u)) continue;
        const int b = mv_of(e);
        const int slot = S.near_base[lo] + (f - S.near_pre[lo]);
        const double4 s = gload(R.pool4 + slot);
        const int sid = gload(R.pidx + slot);
        const int ion = MV.ion[b];
        if (((e & kMbIon) && sid == ion) || ((e & kMbImg) && sid == n_ion + ion)) continue;
        const int t = 2 * b + tb;
        const double dx = MV.tx[t] - s.x, dy = MV.ty[t] - s.y, dz = MV.tz[t] - s.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (tb == 1 && sid < n_ion && sid != ion && d2 <= R.tau2) record_overlap(MV, b, sid, n_ion);
        if (d2 == 0.0) {
            if (!(tb == 1 && sid < n_ion)) record_overlap(MV, b, sid, n_ion);
            continue;
        }
        add_to_t<kBM>(acc, b, s.w * rsqrt_nr(d2));
    }
}

// Hard cores below the far cells of new positions: every cell whose cube comes
// within tau (plus a rounding margin) of the new position is descended.
template <int BLOCK>
__device__ void overlap_below_far_mb(const Rep& R, BTrav<BLOCK>& S, BMoves& MV) {
    using TS = BTrav<BLOCK>;
    const double reach2 = R.reach2;
    int cur = 0, fs = S.n_ovl < TS::OVLCAP ? S.n_ovl : TS::OVLCAP;
    for (int j = threadIdx.x; j < fs; j += BLOCK) S.front[0][j] = S.ovl[j];
    while (fs > 0) {
        if (threadIdx.x == 0) S.cnt2[cur ^ 1] = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < fs; j += BLOCK) {
            const uint32_t e = S.front[cur][j];
            const int c = (int)(e & kCellMask), b = mv_of(e), t = 2 * b + 1;
            const double x = MV.tx[t], y = MV.ty[t], z = MV.tz[t];
            if (c >= R.ncell) { S.err = kErrOvlLeaf; continue; }
            const int4 m = gload(R.cm + c);
            if (m.y >= 0 && m.y + 8 > R.ncell) { S.err = kErrChildLink; continue; }
            if (m.y < 0) {
                if (m.x < 0 || m.z < 0 || m.z + m.x > R.pool) { S.err = kErrOvlLeaf; continue; }
                for (int k = 0; k < m.x; ++k) {
                    const int sid = gload(R.pidx + m.z + k);
                    if (sid >= R.n || sid == MV.ion[b]) continue;
                    const double4 s = gload(R.pool4 + m.z + k);
                    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
                    if (dx * dx + dy * dy + dz * dz <= R.tau2) record_overlap(MV, b, sid, R.n);
                }
            } else {
                for (int d = 0; d < 8; ++d) {
                    const int ch = m.y + d;
                    if (gload(R.cm + ch).x == 0) continue;
                    if (box_dist2(gload(R.cgeo + ch), x, y, z) <= reach2) {
                        const int slot = atomicAdd(&S.cnt2[cur ^ 1], 1);
                        if (slot < TS::FCAP) S.front[cur ^ 1][slot] = (uint32_t)ch | ((uint32_t)b << kMvSh);
                        else S.err = kErrStack;
                    }
                }
            }
        }
        __syncthreads();
        fs = S.cnt2[cur ^ 1];
        if (fs > TS::FCAP) fs = TS::FCAP;
        cur ^= 1;
        __syncthreads();
    }
}

// The traversal of every target of the round from the fs0 entries of level level0 in
// front[0] (as traverse_mc, the two targets of a move sharing an entry); on return
// MV.pot[t] holds target t's potential.  N_0 = 0: a cell holding a remaining source
// is far if it passes the MAC, else opened if it has children, else summed directly.
template <int BLOCK, class Hook>
__device__ void traverse_mb(const Rep& R, BTrav<BLOCK>& S, BMoves& MV, Hook&& hook) {
    using TS = BTrav<BLOCK>;
    constexpr int NW = TS::NW;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    double acc[kBM];  // this lane's target (its parity) of every move
#pragma unroll
    for (int k = 0; k < kBM; ++k) acc[k] = 0.0;
    int cur = 0, fs = MV.fs0, far_n = 0, near_n = 0, nflag = 0, buf = 0;
    bool failed = false, frontier_full = false;
    uint32_t* const gfr = spill_region(R);
    const int gcap = gfr ? (int)(R.spill_words / 2 < 0x7FFFFFFF ? R.spill_words / 2 : 0x7FFFFFFF) : 0;
    const int lcap = R.fcap < TS::FCAP ? R.fcap : TS::FCAP;
    bool rg = false, wg = false;
    PHASE_START();
    for (int level = MV.level0; fs > 0 && !failed; ++level) {
        int next_n = 0;
        // a chunk is kChunk entries per lane: every lane issues the cell loads of all its
        // entries before classifying any, so their latencies overlap and a wide level takes
        // fewer barriers; outputs keep the order of the entries
        for (int base = 0; base < fs; base += kChunk * BLOCK) {
            if (far_n > TS::FARCAP - kChunk * BLOCK) {
                __syncthreads();
                far_pass_mb<BLOCK>(R, S, MV, far_n, 0, acc);
                far_n = 0;
                __syncthreads();
            }
            if (near_n > TS::NEARCAP - kChunk * BLOCK) {
                __syncthreads();
                const int total = near_scan_mb<BLOCK>(S, near_n);
                near_pass_mb<BLOCK>(R, S, MV, near_n, total, acc);
                near_n = 0;
                __syncthreads();
            }
            uint32_t e[kChunk];
            int4 m[kChunk];
            double4 g[kChunk];
            bool valid[kChunk];
#pragma unroll
            for (int h = 0; h < kChunk; ++h) {
                const int j = base + h * BLOCK + tid;
                valid[h] = j < fs;
                e[h] = valid[h] ? (rg ? gfr[(size_t)cur * gcap + j] : S.front[cur][j]) : 0u;
                m[h] = make_int4(0, -1, 0, 0);
                g[h] = make_double4(0.0, 0.0, 0.0, 0.0);
                const int c = (int)(e[h] & kCellMask);
                if (valid[h] && c < R.ncell) { m[h] = gload(R.cm + c); g[h] = gload(R.cgeo + c); }
            }
            if (base == 0) hook(level);
            uint32_t farb[kChunk], nearb[kChunk], copen[kChunk];
            uint64_t bf[kChunk], bn[kChunk], bs[kChunk], bg[kChunk];
            const uint64_t lt = lanemask_lt();
#pragma unroll
            for (int h = 0; h < kChunk; ++h) {
                const int c = (int)(e[h] & kCellMask), b = mv_of(e[h]);
                const int fi = (e[h] & kMbIon) ? 1 : 0, fk = (e[h] & kMbImg) ? 1 : 0;
                const uint32_t open = (e[h] >> kOpSh) & 3u;
                farb[h] = 0; nearb[h] = 0; copen[h] = 0;
                if (valid[h] && c >= R.ncell) {
                    S.err = kErrFrontCell;
                } else if (valid[h]) {
                    const int np = m[h].x - fi - fk;
                    if (m[h].y >= 0 && m[h].y + 8 > R.ncell) {
                        S.err = kErrChildLink;
                    } else if (np > 0) {
                        const int t0 = 2 * b;
                        const double4 gg = g[h];
                        const double dx0 = gg.x - MV.tx[t0], dy0 = gg.y - MV.ty[t0], dz0 = gg.z - MV.tz[t0];
                        const double dx1 = gg.x - MV.tx[t0 + 1], dy1 = gg.y - MV.ty[t0 + 1], dz1 = gg.z - MV.tz[t0 + 1];
                        const double d20 = dx0 * dx0 + dy0 * dy0 + dz0 * dz0;
                        const double d21 = dx1 * dx1 + dy1 * dy1 + dz1 * dz1;
                        const double h2 = 3.0 * (gg.w * gg.w);
                        const uint32_t mac = (h2 <= R.theta2 * d20 ? 1u : 0u) | (h2 <= R.theta2 * d21 ? 2u : 0u);
                        const bool internal = m[h].y >= 0;
                        farb[h] = open & mac;
                        const uint32_t rest = open & ~farb[h];
                        copen[h] = internal ? rest : 0u;
                        nearb[h] = internal ? 0u : rest;
                        if ((farb[h] & 2u) && box_dist2(gg, MV.tx[t0 + 1], MV.ty[t0 + 1], MV.tz[t0 + 1]) <= R.reach2) {
                            const int slot = atomicAdd(&S.n_ovl, 1);
                            if (slot < TS::OVLCAP) S.ovl[slot] = (uint32_t)c | ((uint32_t)b << kMvSh); else S.err = kErrStack;
                        }
                    }
                }
                const bool flagged = (fi | fk) != 0;
                bf[h] = __ballot(farb[h] && !flagged);
                bg[h] = __ballot(farb[h] && flagged);
                bn[h] = __ballot(nearb[h] != 0);
                bs[h] = __ballot(copen[h] != 0);
#ifdef BHMC_PHASE_TIMERS
                {
                    const uint64_t bv = __ballot(valid[h]), be = __ballot(valid[h] && m[h].x - fi - fk <= 0);
                    if (lane == 0) {
                        atomicAdd(&s_phase[kPhEntries], (unsigned long long)__popcll(bv));
                        atomicAdd(&s_phase[kPhEmpty], (unsigned long long)__popcll(be));
                        atomicAdd(&s_phase[kPhFarN], (unsigned long long)(__popcll(bf[h]) + __popcll(bg[h])));
                        atomicAdd(&s_phase[kPhNearN], (unsigned long long)__popcll(bn[h]));
                    }
                }
#endif
                if (lane == 0)
                    S.wcnt[buf][h][w] = (uint64_t)__popcll(bf[h]) | ((uint64_t)__popcll(bn[h]) << 16) |
                                        ((uint64_t)__popcll(bs[h]) << 32) | ((uint64_t)__popcll(bg[h]) << 48);
            }
            PHASE_COUNT(kPhChunks, 1);
            __syncthreads();
            // offsets: the entries of part h of every wave come after all of part h - 1
            uint64_t before[kChunk], tot[kChunk];
#pragma unroll
            for (int h = 0; h < kChunk; ++h) {
                before[h] = 0; tot[h] = 0;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) {
                    const uint64_t v = S.wcnt[buf][h][ww];
                    before[h] += ww < w ? v : 0ull;
                    tot[h] += v;
                }
            }
            buf ^= 1;
            uint64_t all = 0;
#pragma unroll
            for (int h = 0; h < kChunk; ++h) all += tot[h];
            const int tf = (int)(all & 0xffff), tn = (int)((all >> 16) & 0xffff);
            const int ts = (int)((all >> 32) & 0xffff), tg = (int)(all >> 48);
            if (nflag + tg > 4 * kBM) {  // uniform
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
            uint64_t prior = 0;  // the parts before h, summed over the whole workgroup
#pragma unroll
            for (int h = 0; h < kChunk; ++h) {
                const uint64_t at = prior + before[h];
                prior += tot[h];
                const int c = (int)(e[h] & kCellMask), b = mv_of(e[h]);
                const int fi = (e[h] & kMbIon) ? 1 : 0, fk = (e[h] & kMbImg) ? 1 : 0;
                const bool flagged = (fi | fk) != 0;
                const uint32_t flags = e[h] & (kMbIon | kMbImg);
                const uint32_t mvb = (uint32_t)b << kMvSh;
                if (farb[h] && !flagged)
                    S.farl[far_n + (int)(at & 0xffff) + __popcll(bf[h] & lt)] = (uint32_t)c | mvb | (farb[h] << kOpSh);
                if (farb[h] && flagged)
                    S.flagl[nflag + (int)(at >> 48) + __popcll(bg[h] & lt)] = (uint32_t)c | mvb | (farb[h] << kOpSh) | flags;
                if (nearb[h]) {
                    const int o = near_n + (int)((at >> 16) & 0xffff) + __popcll(bn[h] & lt);
                    S.nearl[o] = (uint32_t)c | mvb | (nearb[h] << kOpSh) | flags;
                    S.near_base[o] = m[h].z;
                    S.near_pre[o] = m[h].x;
                    if (m[h].x < 0 || m[h].z < 0 || m[h].z + m[h].x > R.pool) { S.near_pre[o] = 0; S.err = kErrNearSlots; }
                }
                if (copen[h]) {
                    const int o = next_n + 8 * ((int)((at >> 32) & 0xffff) + __popcll(bs[h] & lt));
                    const int dig_i = fi ? key_digit(MV.key[b][0], level + 1) : -1;
                    const int dig_k = fk ? key_digit(MV.key[b][2], level + 1) : -1;
                    const uint32_t hdr = mvb | (copen[h] << kOpSh);
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        const uint32_t fl = (d == dig_i ? kMbIon : 0u) | (d == dig_k ? kMbImg : 0u);
                        const uint32_t ne = (uint32_t)(m[h].y + d) | hdr | fl;
                        if (wg) gfr[(size_t)(cur ^ 1) * gcap + o + d] = ne;
                        else S.front[cur ^ 1][o + d] = ne;
                    }
                }
            }
            far_n += tf; near_n += tn; nflag += tg; next_n += 8 * ts;
        }
        __syncthreads();
        cur ^= 1;
        fs = next_n;
        rg = wg;
    }
    PHASE(kPhLevels);
    if (failed) {
        if (tid == 0) S.err = frontier_full ? kErrFrontier : kErrStack;
        __syncthreads();
        return;
    }
    // corrected moments of the far cells that hold a mover's own ion or image
    for (int it = tid; it < nflag * NTERM; it += BLOCK) {
        const int f = it / NTERM, k = it % NTERM;
        const uint32_t e = S.flagl[f];
        const int c = (int)(e & kCellMask), b = mv_of(e);
        if (c >= R.ncell) { S.err = kErrFlagCell; S.Mx[f][k] = 0.0; continue; }
        const double4 g = R.cgeo[c];
        double mk = R.M[(size_t)c * MSTR + k];
        if (e & kMbIon) { const double4 s = MV.ct[b][0]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        if (e & kMbImg) { const double4 s = MV.ct[b][2]; mk = mk - s.w * mono(S.mi[k], s.x - g.x, s.y - g.y, s.z - g.z); }
        S.Mx[f][k] = mk;
    }
    const int total = near_scan_mb<BLOCK>(S, near_n);  // its barriers also publish Mx
    PHASE(kPhFlagged);
    far_pass_mb<BLOCK>(R, S, MV, far_n, nflag, acc);
#ifdef BHMC_PHASE_TIMERS
    __syncthreads();
    PHASE(kPhFar);
#endif
    near_pass_mb<BLOCK>(R, S, MV, near_n, total, acc);
#pragma unroll
    for (int k = 0; k < kBM; ++k) {
        const double sum = wave_sum_parity(acc[k]);
        if (lane < 2) S.red[w][2 * k + lane] = sum;
    }
    __syncthreads();
    PHASE(kPhNear);
    if (S.n_ovl > 0 && S.err == 0) overlap_below_far_mb<BLOCK>(R, S, MV);
    PHASE(kPhOverlap);
    if (tid < kBT) {
        double sum = 0.0;
        for (int ww = 0; ww < NW; ++ww) sum += S.red[ww][tid];
        MV.pot[tid] = sum;
    }
}

// What contribution cc of move j adds (per unit charge) to the potential at x through
// the tree: walk its root path from the top; the first cell passing the MAC takes it
// through its expansion, otherwise its leaf takes it directly.
__device__ __forceinline__ double path_value(const Rep& R, const BMoves& MV, int j, int cc, double x, double y, double z) {
    const double4 src = MV.ct[j][cc];
    const int len = MV.plen[j][cc];
    for (int l = 0; l < len; ++l) {
        const double4 g = MV.path_geo[j][cc][l];
        const double dx = g.x - x, dy = g.y - y, dz = g.z - z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (3.0 * (g.w * g.w) <= R.theta2 * d2) return point_expansion(dx, dy, dz, src.x - g.x, src.y - g.y, src.z - g.z);
    }
    const double dx = x - src.x, dy = y - src.y, dz = z - src.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    return d2 == 0.0 ? 0.0 : rsqrt_nr(d2);
}

struct RoundOut { int done; int stop; int detail; };

// One stage of the commit prefetch of move b's ion (j = 0) or image (j = 1).
__device__ __forceinline__ void prefetch_stage_mb(const Rep& R, BMoves& MV, int b, int j) {
    const int s = j == 0 ? MV.ion[b] : R.n + MV.ion[b];
    const int stage = MV.pf_stage[b][j];
    if (stage == 0) {
        const int2 t = gload(R.track + s);
        MV.tr[b][j] = t;
        MV.pf_stage[b][j] = (t.x >= 0 && t.x < R.ncell) ? 1 : 9;
    } else if (stage == 1) {
        const int4 m = gload(R.cm + MV.tr[b][j].x);
        MV.lm_old[b][j] = m;
        const bool sane = m.y < 0 && m.x >= 1 && m.z >= 0 && m.z + m.x <= R.pool && m.x <= m.w &&
                          MV.tr[b][j].y >= 0 && MV.tr[b][j].y < m.x;
        MV.pf_stage[b][j] = sane ? 2 : 9;
    } else if (stage == 2) {
        const int4 m = MV.lm_old[b][j];
        MV.last_pidx[b][j] = gload(R.pidx + m.z + m.x - 1);
        MV.last_pool[b][j] = gload(R.pool4 + m.z + m.x - 1);
        MV.self_pidx[b][j] = gload(R.pidx + m.z + MV.tr[b][j].y);
        MV.pf_stage[b][j] = 3;
    }
}

// One round of up to nb moves (draws b0 .. b0 + nb - 1 of MV's batch, move indices
// m .. m + nb - 1).  Returns the number of moves consumed and a stop status.
template <int BLOCK>
__device__ RoundOut round_mb(const Rep& R, BTrav<BLOCK>& S, BMoves& MV, int b0, int nb) {
    static_assert(BLOCK >= 256, "the path descents and the commit prefetch run on the last two waves");
    const int tid = threadIdx.x;
    const bool imgs = R.images != 0;
    const int nps = imgs ? 4 : 2;
    PHASE_START();
    // ---- set-up: lane 4b + j prepares contribution j of move b
    if (tid < 4 * nb) {
        const int b = tid >> 2, j = tid & 3;
        const int i = MV.dr_i[b0 + b];
        const double4 si = gload(R.src + i);
        const double4 mo = imgs ? gload(R.src + R.n + i) : make_double4(0, 0, 0, 0);
        const double rx = si.x + MV.dr_d[b0 + b][0], ry = si.y + MV.dr_d[b0 + b][1], rz = si.z + MV.dr_d[b0 + b][2];
        double4 cj;
        if (j == 0) cj = si;
        else if (j == 1) cj = make_double4(rx, ry, rz, si.w);
        else if (j == 2) cj = mo;
        else cj = imgs ? kelvin(R, rx, ry, rz, si.w) : make_double4(0, 0, 0, 0);
        MV.ct[b][j] = cj;
        MV.key[b][j] = (j < 2 || imgs) ? morton_key(R, cj.x, cj.y, cj.z) : 0;
        if (j == 0) {
            MV.ion[b] = i;
            MV.alpha[b] = MV.dr_d[b0 + b][3];
            MV.wall[b] = outside(R, rx, ry, rz) ? 1 : 0;
            MV.tx[2 * b] = si.x; MV.ty[2 * b] = si.y; MV.tz[2 * b] = si.z;
            MV.tx[2 * b + 1] = rx; MV.ty[2 * b + 1] = ry; MV.tz[2 * b + 1] = rz;
            MV.ovl_fixed[b] = 0;
            MV.ovl_moved[b] = 0u;
            MV.ovl_new[b] = 0u;
            MV.acc[b] = 0;
            MV.reason[b] = 0;
        }
    }
    if (tid == 0) {
        MV.nb = nb;
        S.n_ovl = 0; S.err = 0;
        MV.err = 0; MV.nlist = 0; MV.stop = 0; MV.ndone = 0;
        // the root holds every target, so the MAC never takes it: with more than N_0 = 0
        // sources besides a move's own two it is opened and the traversal starts at level 1
        const int np_root = R.nsrc - 1 - (imgs ? 1 : 0);
        MV.level0 = (R.ncell > 1 && np_root > 0) ? 1 : 0;
    }
    const int th = tid - (BLOCK - 64), tp = tid - (BLOCK - 128);
    if (th >= 0 && th < 4 * nb) { MV.path[th >> 2][th & 3][0] = 0; MV.plen[th >> 2][th & 3] = 0; }
    if (tp >= 0 && tp < 2 * nb) MV.pf_stage[tp >> 1][tp & 1] = ((tp & 1) && !imgs) ? 3 : 0;
    __syncthreads();
    // first frontier: the eight children of the root (or the root) for every move inside the walls
    if (tid < 8 * nb) {
        const int b = tid >> 3, d = tid & 7;
        if (!MV.wall[b]) {
            int before = 0;
            for (int bb = 0; bb < b; ++bb) before += MV.wall[bb] ? 0 : 1;
            const uint32_t hdr = ((uint32_t)b << kMvSh) | (3u << kOpSh);
            if (MV.level0 == 1) {
                const int di = key_digit(MV.key[b][0], 1), dk = imgs ? key_digit(MV.key[b][2], 1) : -1;
                S.front[0][8 * before + d] = (uint32_t)(1 + d) | hdr | (d == di ? kMbIon : 0u) | (d == dk ? kMbImg : 0u);
            } else if (d == 0) {
                S.front[0][before] = hdr | kMbIon | (imgs ? kMbImg : 0u);
            }
        }
    }
    if (tid == 0) {
        int act = 0;
        for (int b = 0; b < nb; ++b) act += MV.wall[b] ? 0 : 1;
        MV.fs0 = MV.level0 == 1 ? 8 * act : act;
    }
    int my_level = 0;
    const int pb = th >> 2, pj = th & 3;
    const bool path_lane = th >= 0 && th < 4 * nb && pj < nps && !MV.wall[pb];
    const bool pf_lane = tp >= 0 && tp < 2 * nb && !MV.wall[tp >> 1];
    __syncthreads();
    auto step = [&](int level) {
        const int c = MV.path[pb][pj][level];
        const bool cok = c >= 0 && c < R.ncell;
        const int link = cok ? gload(R.cm + c).y : -1;
        if (cok) MV.path_geo[pb][pj][level] = gload(R.cgeo + c);
        if (c < 0 || c >= R.ncell || (link >= 0 && link + 8 > R.ncell)) {
            MV.err = kErrPathCell;
            MV.plen[pb][pj] = level + 1;
            MV.path[pb][pj][level] = 0;
        } else if (link >= 0 && level + 1 < kMaxLevels) {
            MV.path[pb][pj][level + 1] = link + key_digit(MV.key[pb][pj], level + 1);
        } else {
            if (link >= 0) MV.err = kErrPathDepth;
            MV.plen[pb][pj] = level + 1;
            if (pj & 1) {  // a new position's leaf: its slot state for the commit
                const int4 m = gload(R.cm + c);
                MV.lm_new[pb][pj >> 1] = m;
                if (m.y >= 0 || m.z < 0 || m.x < 0 || m.z + m.w > R.pool) MV.err = kErrCommitLeaf;
            }
        }
    };
    auto hook = [&](int) {
#ifdef BHMC_PHASE_TIMERS
        const long long hk0 = wall_clock64();
#endif
        if (path_lane)
            for (int k = 0; k < 2 && MV.plen[pb][pj] == 0 && my_level < kMaxLevels; ++k) step(my_level++);
#ifdef BHMC_PHASE_TIMERS
        const long long hk1 = wall_clock64();
        if (th == 0) atomicAdd(&s_phase[kPhHookPath], (unsigned long long)(hk1 - hk0));
#endif
        if (pf_lane)
            for (int k = 0; k < 2; ++k) prefetch_stage_mb(R, MV, tp >> 1, tp & 1);
#ifdef BHMC_PHASE_TIMERS
        if (tp == 0) atomicAdd(&s_phase[kPhHookPf], (unsigned long long)(wall_clock64() - hk1));
#endif
    };
    PHASE(kPhSetup);
    traverse_mb<BLOCK>(R, S, MV, hook);
#ifdef BHMC_PHASE_TIMERS
    ph_t0_ = wall_clock64();
#endif
    if (S.err) {
        RoundOut o{0, (S.err == kErrStack || S.err == kErrFrontier) ? -7 : -8, S.err};
        __syncthreads();
        return o;
    }
    if (path_lane) {
        while (MV.plen[pb][pj] == 0 && my_level < kMaxLevels) step(my_level++);
        if (MV.plen[pb][pj] == 0) { MV.err = kErrPathDepth; MV.plen[pb][pj] = 1; MV.path[pb][pj][0] = 0; }
    }
    if (pf_lane) {
        for (int k = 0; k < 3 && MV.pf_stage[tp >> 1][tp & 1] < 3; ++k) prefetch_stage_mb(R, MV, tp >> 1, tp & 1);
        if (MV.pf_stage[tp >> 1][tp & 1] != 3) MV.err = kErrCommitSlot;
    }
    __syncthreads();
    PHASE(kPhPaths);
    if (MV.err) {
        RoundOut o{0, -8, MV.err};
        __syncthreads();
        return o;
    }
    // ---- in parallel (threads 0-127, 128-191, 192-199): corrections (thread (j, b, t), j < b: what move j's four contributions add
    // to target t of move b once j is committed); for every pair, whether b's new position
    // overlaps j's and how j changes the counts of b's new leaves; for every move, its energy
    // change on the start-of-round tree and whether its tracked leaves are the ones its keys
    // lead to
    if (tid < 2 * nb * nb) {
        const int j = tid / (2 * nb), b = (tid >> 1) % nb, tb = tid & 1;
        if (j < b && !MV.wall[j] && !MV.wall[b]) {
            const int t = 2 * b + tb;
            const double x = MV.tx[t], y = MV.ty[t], z = MV.tz[t];
            double v = 0.0;
            for (int cc = 0; cc < nps; ++cc) {
                const double w = MV.ct[j][cc].w * path_value(R, MV, j, cc, x, y, z);
                v = (cc & 1) ? v + w : v - w;
            }
            MV.corr[j][b][tb] = v;
        }
    } else if (tid >= 128 && tid < 128 + nb * nb) {
        const int j = (tid - 128) / nb, b = (tid - 128) % nb;
        if (j < b && !MV.wall[j] && !MV.wall[b]) {
            const double4 sn = MV.ct[b][1], s = MV.ct[j][1];
            const double dx = sn.x - s.x, dy = sn.y - s.y, dz = sn.z - s.z;
            if (dx * dx + dy * dy + dz * dz <= R.tau2) atomicOr(&MV.ovl_new[b], 1u << j);
            // leaves of the moves: ion old / new, image old / new
            const int cio = MV.tr[j][0].x, cin = MV.path[j][1][MV.plen[j][1] - 1];
            const int cmo = imgs ? MV.tr[j][1].x : -1, cmn = imgs ? MV.path[j][3][MV.plen[j][3] - 1] : -1;
            const int bin = MV.path[b][1][MV.plen[b][1] - 1];
            const int bmn = imgs ? MV.path[b][3][MV.plen[b][3] - 1] : -2;
            int ei = 0, em = 0;
            if (cin != cio) { ei += (cin == bin) - (cio == bin); em += (cin == bmn) - (cio == bmn); }
            if (imgs && cmn != cmo) { ei += (cmn == bin) - (cmo == bin); em += (cmn == bmn) - (cmo == bmn); }
            MV.e_ion[b][j] = ei;
            MV.e_img[b][j] = em;
        }
    } else if (tid >= 192 && tid < 192 + nb) {
        const int b = tid - 192;
        if (!MV.wall[b]) {
            const double4 sn = MV.ct[b][1], so = MV.ct[b][0];
            const double q = so.w, l = R.l_B;
            double d0 = 0.0;  // the exact self-image and central-charge changes
            if (R.geom == 1) {
                const double rn2 = sn.x * sn.x + sn.y * sn.y + sn.z * sn.z;
                const double ro2 = so.x * so.x + so.y * so.y + so.z * so.z;
                if (imgs) d0 += 0.5 * l * R.gamma * R.a * q * q * (1.0 / (rn2 - R.a2) - 1.0 / (ro2 - R.a2));
                if (R.Qc != 0.0) d0 += l * R.Qc * q * (1.0 / sqrt(rn2) - 1.0 / sqrt(ro2));
            }
            MV.dE0[b] = d0;
            bool sane = MV.tr[b][0].x == MV.path[b][0][MV.plen[b][0] - 1];
            if (imgs) sane = sane && MV.tr[b][1].x == MV.path[b][2][MV.plen[b][2] - 1];
            MV.sane[b] = sane ? 1 : 0;
        }
    }
    __syncthreads();
    PHASE(kPhCorr);
    // ---- decisions, in move order, by the first wave.  Lane b holds everything move b needs,
    // what every earlier move of the round adds to it included, so deciding move b is lane b's
    // own arithmetic on the mask of the moves accepted so far; one read of that lane's verdict
    // then updates the mask for the next move.
    if (tid < 64) {
        const int lane = tid;
        const bool mine = lane < nb;
        double cr0[kBM], cr1[kBM];
        int ei_r[kBM], em_r[kBM];
#pragma unroll
        for (int j = 0; j < kBM; ++j) {
            const bool v = mine && j < lane;
            cr0[j] = v ? MV.corr[j][lane][0] : 0.0;
            cr1[j] = v ? MV.corr[j][lane][1] : 0.0;
            ei_r[j] = v ? MV.e_ion[lane][j] : 0;
            em_r[j] = v ? MV.e_img[lane][j] : 0;
        }
        const int my_wall = mine ? MV.wall[lane] : 1;
        const int my_fixed = mine ? MV.ovl_fixed[lane] : 0;
        const uint32_t my_moved = mine ? MV.ovl_moved[lane] : 0u, my_new = mine ? MV.ovl_new[lane] : 0u;
        const double my_pn = mine ? MV.pot[2 * lane + 1] : 0.0, my_po = mine ? MV.pot[2 * lane] : 0.0;
        const double my_q = mine ? MV.ct[lane][0].w : 0.0, my_d0 = mine ? MV.dE0[lane] : 0.0;
        const double my_alpha = mine ? MV.alpha[lane] : 0.0;
        const int my_sane = mine ? MV.sane[lane] : 0;
        const int my_cio = mine ? MV.tr[lane][0].x : -1;
        const int my_cin = mine ? MV.path[lane][1][MV.plen[lane][1] - 1] : -1;
        const int my_cmo = (mine && imgs) ? MV.tr[lane][1].x : -1;
        const int my_cmn = (mine && imgs) ? MV.path[lane][3][MV.plen[lane][3] - 1] : -1;
        const int4 my_l0 = mine ? MV.lm_new[lane][0] : make_int4(0, 0, 0, 0);
        const int4 my_l1 = (mine && imgs) ? MV.lm_new[lane][1] : make_int4(0, 0, 0, 0);
        uint32_t acc_mask = 0;
        int done = nb, stop = 0, err = 0;
        int my_reason = 0, my_acc = 0;
        double my_dE = kInf;
        bool ended = false;
#pragma unroll
        for (int b = 0; b < kBM; ++b) {
            if (b >= nb || ended) continue;  // uniform
            // verdict of lane b: bit 0 accepted, bit 1 its commit would overflow a leaf index
            // array, bit 2 its tracked leaves are not where its keys lead
            int out = 0, reason = 0;
            double dE = kInf;
            if (lane == b) {
                if (my_wall) {
                    reason = 1;
                } else if (my_fixed != 0 || (my_moved & ~acc_mask) != 0u || (my_new & acc_mask) != 0u) {
                    reason = 2;
                } else {
                    double c1 = 0.0, c0 = 0.0;
                    int ei = 0, em = 0;
#pragma unroll
                    for (int j = 0; j < kBM; ++j)
                        if (j < b && ((acc_mask >> j) & 1u)) { c1 += cr1[j]; c0 += cr0[j]; ei += ei_r[j]; em += em_r[j]; }
                    const double pn = my_pn + c1, po = my_po + c0;
                    dE = R.l_B * my_q * (pn - po) + my_d0;
                    if (dE <= 0.0 || my_alpha <= exp(-dE)) {
                        if (!my_sane) {
                            out = 4;
                        } else {
                            // would a leaf index array overflow?
                            bool ok = !(my_cin != my_cio && my_l0.x + ei + 1 > my_l0.w);
                            if (imgs && my_cmn != my_cmo) {
                                int c = my_l1.x + em;
                                if (my_cin != my_cio) { if (my_cmn == my_cin) c += 1; if (my_cmn == my_cio) c -= 1; }
                                if (c + 1 > my_l1.w) ok = false;
                            }
                            out = ok ? 1 : 2;
                        }
                    }
                }
            }
            out = __builtin_amdgcn_readlane(out, b);  // uniform from here
            if (out & 4) { err = kErrCommitSlot; done = b; ended = true; continue; }
            if (out & 2) { stop = -6; done = b; ended = true; continue; }
            if (out & 1) acc_mask |= 1u << b;
            if (lane == b) { my_reason = reason; my_dE = dE; my_acc = out & 1; }
        }
        if (mine) {
            MV.reason[lane] = my_reason;
            MV.dE[lane] = my_dE;
            MV.acc[lane] = (lane < done) ? my_acc : 0;
        }
        if (lane == 0) { MV.ndone = done; MV.stop = stop; MV.err = err; }
        // the leaf index array operations of the accepted moves: lane 4b + k, k = ion old, ion new,
        // image old, image new (in this order, the order of the move-by-move commit)
        if (lane < 4 * kBM) {
            const int b = lane >> 2, k = lane & 3;
            int type = 0, cell = -1, src = -1, slot0 = -1;
            int4 hdr = make_int4(0, 0, 0, 0);
            if (b < done && ((acc_mask >> b) & 1u) && (k < 2 || imgs)) {
                const int j = k >> 1;  // 0: the ion, 1: the image
                const int c_old = MV.tr[b][j].x, c_new = MV.path[b][2 * j + 1][MV.plen[b][2 * j + 1] - 1];
                src = j == 0 ? MV.ion[b] : R.n + MV.ion[b];
                if (c_old == c_new) {
                    if ((k & 1) == 0) { type = 3; cell = c_old; hdr = MV.lm_old[b][j]; slot0 = MV.tr[b][j].y; }
                } else if ((k & 1) == 0) {
                    type = 1; cell = c_old; hdr = MV.lm_old[b][j]; slot0 = MV.tr[b][j].y;
                } else {
                    type = 2; cell = c_new; hdr = MV.lm_new[b][j];
                }
            }
            MV.op_type[lane] = type;
            MV.op_cell[lane] = cell;
            MV.op_src[lane] = src;
            MV.op_slot[lane] = slot0;
            MV.op_base[lane] = hdr.z;
            MV.op_count[lane] = hdr.x;
        }
    }
    __syncthreads();
    PHASE(kPhDecide);
    if (MV.err) {
        RoundOut o{0, -8, MV.err};
        __syncthreads();
        return o;
    }
    const int ndone = MV.ndone;
    // ---- leaf index arrays (Sec. 3.3: delete = the last entry fills the hole, add = append), one
    // lane per leaf taking that leaf's operations in order; moves between leaves are independent.
    // A source that fills a hole and leaves the leaf later in the round has its slot followed in
    // op_slot; its final tracking is written by the lane of the leaf it moves to.
    if (tid < 64) {
        // lane o < 4 kBM holds operation o; the loops below walk the operations in order, the
        // same for every lane, reading each one's fields from its lane
        const int o = tid;
        const bool has = o < 4 * kBM;
        const int my_type = has ? MV.op_type[o] : 0;
        const int my_cell = has ? MV.op_cell[o] : -1;
        const int my_src = has ? MV.op_src[o] : -1;
        const int base = has ? MV.op_base[o] : 0;
        int count = has ? MV.op_count[o] : 0;
        bool lead = my_type != 0;
#pragma unroll
        for (int o2 = 0; o2 < 4 * kBM; ++o2) {
            const int t2 = __builtin_amdgcn_readlane(my_type, o2), c2 = __builtin_amdgcn_readlane(my_cell, o2);
            if (o2 < o && t2 != 0 && c2 == my_cell) lead = false;
        }
        bool touched = false;  // an earlier operation of the round has changed this leaf
        for (int o2 = 0; o2 < 4 * kBM; ++o2) {
            const int type = __builtin_amdgcn_readlane(my_type, o2);
            if (type == 0) continue;  // uniform
            const int cell = __builtin_amdgcn_readlane(my_cell, o2);
            const int src = __builtin_amdgcn_readlane(my_src, o2);
            if (!lead || cell != my_cell) continue;
            const double4 nv = MV.ct[o2 >> 2][(o2 & 3) == 0 || (o2 & 3) == 1 ? 1 : 3];
            if (type == 2) {  // append
                R.pool4[base + count] = nv;
                R.pidx[base + count] = src;
                R.track[src] = make_int2(cell, count);
                ++count;
            } else {
                const int k = MV.op_slot[o2];
                if (type == 3) {  // the source stays in this leaf: new position in place
                    R.pool4[base + k] = nv;
                } else {          // delete: the last entry fills the hole
                    const int last = count - 1;
                    if (k != last) {
                        // untouched, the leaf is as it was when its last entry was prefetched
                        const int jb = o2 >> 2, jj = (o2 & 3) >> 1;
                        const int moved = touched ? R.pidx[base + last] : MV.last_pidx[jb][jj];
                        const double4 mv = touched ? R.pool4[base + last] : MV.last_pool[jb][jj];
                        R.pool4[base + k] = mv;
                        R.pidx[base + k] = moved;
                        bool leaves_later = false;
                        for (int o3 = o2 + 1; o3 < 4 * kBM; ++o3)
                            if (MV.op_cell[o3] == cell && (MV.op_type[o3] == 1 || MV.op_type[o3] == 3) &&
                                MV.op_src[o3] == moved) {
                                MV.op_slot[o3] = k;
                                leaves_later = MV.op_type[o3] == 1;
                            }
                        if (moved < 0 || moved >= R.nsrc) MV.err = kErrCommitSource;
                        else if (!leaves_later) R.track[moved] = make_int2(cell, k);
                    }
                    count = last;
                }
            }
            if (type != 1) R.src[src] = nv;
            touched = true;
        }
        if (lead) R.cm[my_cell].x = count;
    }
    // ---- meanwhile, on the other waves: distinct cells of the accepted moves' root paths, in
    // (move, contribution) order, each with the contributions that apply to it
    for (int it = tid - 64; it < ndone * 4 * kMaxLevels; it += BLOCK - 64) {
        if (it < 0) break;  // the first wave (leaf index arrays above)
        const int j = it / (4 * kMaxLevels), cc = (it / kMaxLevels) & 3, l = it % kMaxLevels;
        if (!MV.acc[j] || cc >= nps || l >= MV.plen[j][cc]) continue;
        const int c = MV.path[j][cc][l];
        bool owner = true;
        for (int jj = 0; jj <= j && owner; ++jj) {
            if (!MV.acc[jj]) continue;
            const int cmax = jj < j ? nps : cc;
            for (int c2 = 0; c2 < cmax; ++c2)
                if (l < MV.plen[jj][c2] && MV.path[jj][c2][l] == c) { owner = false; break; }
        }
        if (!owner) continue;
        uint32_t mask = 0;
        for (int jj = j; jj < ndone; ++jj) {
            if (!MV.acc[jj]) continue;
            for (int c2 = (jj == j ? cc : 0); c2 < nps; ++c2)
                if (l < MV.plen[jj][c2] && MV.path[jj][c2][l] == c) mask |= 1u << (4 * jj + c2);
        }
        const int slot = atomicAdd(&MV.nlist, 1);
        MV.list_cell[slot] = c;
        MV.list_mask[slot] = mask;
        MV.list_at[slot] = ((j * 4 + cc) * kMaxLevels + l) | (l < MV.plen[j][cc] - 1 ? (1 << 30) : 0);
    }
    __syncthreads();
    PHASE(kPhSlots);
    // ---- moments and counts of the distinct path cells, contributions in move order.  The powers
    // of each path entry's offset from its cell centre are tabulated first (in the traversal's
    // list space), so a term is three table reads per contribution; without room, d^n is
    // formed by repeated multiplication.
    if (tid < 64) {  // first power-table row of each path entry: an exclusive scan of the path lengths
        const int jc = tid, j = jc >> 2, cc = jc & 3;
        const bool on = jc < 4 * kBM && j < ndone && MV.acc[j] && cc < nps;
        const int len = on ? MV.plen[j][cc] : 0;
        int x = len;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (tid >= off) x += y;
        }
        if (jc < 4 * kBM) MV.pw_row[jc] = on ? x - len : -1;
        if (tid == 63) MV.pw_rows = x;
    }
    __syncthreads();
    const bool use_pw = MV.pw_rows <= BTrav<BLOCK>::PWROWS;
    if (use_pw) {
        for (int it = tid; it < 4 * kBM * kMaxLevels * 3; it += BLOCK) {
            const int jc = it / (kMaxLevels * 3), l = (it / 3) % kMaxLevels, ax = it % 3;
            const int j = jc >> 2, cc = jc & 3;
            if (MV.pw_row[jc] < 0 || l >= MV.plen[j][cc]) continue;
            const double4 sc = MV.ct[j][cc], g = MV.path_geo[j][cc][l];
            const double d = ax == 0 ? sc.x - g.x : (ax == 1 ? sc.y - g.y : sc.z - g.z);
            double* row = S.pw[MV.pw_row[jc] + l][ax];
            double v = 1.0;
            row[0] = 1.0;
            for (int e = 1; e <= P; ++e) { v *= d; row[e] = v; }
        }
        __syncthreads();
    }
    const int items = MV.nlist * NTERM;
    constexpr int G = 4;
    for (int base = tid; base < items; base += G * BLOCK) {
        double mk[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int it = base + u * BLOCK;
            if (it < items) mk[u] = R.M[(size_t)MV.list_cell[it / NTERM] * MSTR + it % NTERM];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int it = base + u * BLOCK;
            if (it >= items) continue;
            const int li = it / NTERM, k = it % NTERM;
            const int c = MV.list_cell[li];
            const int at = MV.list_at[li];
            const int l = (at & ((1 << 30) - 1)) % kMaxLevels;
            const uint32_t code = S.mi[k];
            const int n1 = (int)(code & 255u), n2 = (int)((code >> 8) & 255u), n3 = (int)(code >> 16);
            double m = mk[u];
            int dc = 0;
            for (uint32_t rest = MV.list_mask[li]; rest; rest &= rest - 1u) {
                const int bit = __builtin_ctz(rest);
                const double4 sc = MV.ct[bit >> 2][bit & 3];
                double v;
                if (use_pw) {
                    const int row = MV.pw_row[bit] + l;
                    v = S.pw[row][0][n1] * S.pw[row][1][n2] * S.pw[row][2][n3];
                } else {
                    const double4 g = MV.path_geo[bit >> 2][bit & 3][l];
                    v = mono(code, sc.x - g.x, sc.y - g.y, sc.z - g.z);
                }
                if (bit & 1) { m = m + sc.w * v; ++dc; } else { m = m - sc.w * v; --dc; }
            }
            R.M[(size_t)c * MSTR + k] = m;
            if (R.M32) R.M32[(size_t)c * MSTR + k] = (float)m;
            if (k == 0 && (at & (1 << 30)) && dc != 0) R.cm[c].x += dc;
        }
    }
    __syncthreads();
    PHASE(kPhMoments);
    PHASE_COUNT(kPhRounds, 1);
    PHASE_COUNT(kPhMoves, ndone);
    RoundOut o{ndone, MV.stop, MV.err};
    if (MV.err) o.stop = -8;
    return o;
}

// Persistent Metropolis kernel with batched rounds (same queue, statistics and stop
// protocol as k_mc): each workgroup takes replicas from the queue and advances its
// chain round by round.  A.bm caps the moves per round (at most kBM).
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_mcb(Rep* reps, McArgs A) {
    __shared__ BTrav<BLOCK> S;
    __shared__ BMoves MV;
    __shared__ Rep Rs;
    __shared__ int s_r;
    const int tid = threadIdx.x;
    for (int k = tid; k < NTERM; k += BLOCK) S.mi[k] = mi_code(k);
#ifdef BHMC_PHASE_TIMERS
    for (int k = tid; k < kNumPhases; k += BLOCK) s_phase[k] = 0;
#endif
    const int bmax = A.bm > 0 && A.bm < kBM ? A.bm : kBM;
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
        long long st_moves = 0, st_acc = 0, st_wall = 0, st_ovl = 0, st_met = 0;
        int status = 0, detail = 0;
        while (m < mend) {
            const int b0 = (int)((m - m0) & (kDrawBatch - 1));
            if (b0 == 0) {
                if (tid < kDrawBatch && m + tid < mend) {
                    const Draw d = draw_move(A.seed, (uint32_t)r, (uint64_t)(m + tid), Rs.n, A.step);
                    MV.dr_i[tid] = d.i;
                    MV.dr_d[tid][0] = d.dx; MV.dr_d[tid][1] = d.dy; MV.dr_d[tid][2] = d.dz;
                    MV.dr_d[tid][3] = d.alpha;
                }
                __syncthreads();
            }
            // the round: moves of distinct ions, within the drawn batch and the chain
            long long left = mend - m;
            int nb = bmax;
            if (nb > kDrawBatch - b0) nb = kDrawBatch - b0;
            if ((long long)nb > left) nb = (int)left;
            for (int b = 1; b < nb; ++b) {
                bool rep = false;
                for (int j = 0; j < b; ++j) rep = rep || MV.dr_i[b0 + b] == MV.dr_i[b0 + j];
                if (rep) { nb = b; break; }
            }
            const RoundOut o = round_mb<BLOCK>(Rs, S, MV, b0, nb);
            if (tid == 0) {
                for (int b = 0; b < o.done; ++b) {
                    ++st_moves;
                    if (MV.acc[b]) ++st_acc;
                    else if (MV.reason[b] == 1) ++st_wall;
                    else if (MV.reason[b] == 2) ++st_ovl;
                    else ++st_met;
                    if (A.accept) A.accept[m + b - A.move_base] = (uint8_t)MV.acc[b];
                }
            }
            m += o.done;
            if (o.stop) { status = o.stop; detail = o.detail; break; }
            __syncthreads();
        }
        if (tid == 0) {
            Rep* gr = reps + r;
            gr->move_next = m;
            gr->mc_status = status;
            if (detail) gr->err_detail = detail;
            gr->stats[0] += st_moves; gr->stats[1] += st_acc; gr->stats[2] += st_wall;
            gr->stats[3] += st_ovl; gr->stats[4] += st_met;
#ifdef BHMC_PHASE_TIMERS
            for (int k = 0; k < kNumPhases; ++k) {
                atomicAdd(&g_phase[k], s_phase[k]);
                s_phase[k] = 0;
            }
#endif
        }
        __syncthreads();
    }
}
