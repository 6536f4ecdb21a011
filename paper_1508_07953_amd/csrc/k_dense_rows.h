// k_dense_rows.h -- the row-layout dense search kernels, included by
// k_dense_rows.hip (the default block shape of every patch width, and the
// k-NN variant) and k_dense_rows_shapes.hip (the other block shapes, which
// the autotuner can select at run time).
//
// Exact exhaustive search with references as the MFMA
// rows and queries as the columns (v_mfma_i32_32x32x32_i8), the default dense
// search at every patch width.
//
// With a = 127 - q, v = r - 128 and p = Rc & 1, the per-reference value
// Hf = (Rc + bias - p) / 2 enters as the MFMA's C operand, read straight from
// LDS, so the accumulator is Y = Hf + <a, v> and SSD - Qc + bias = 2Y + p
// exactly.  The references run in the index's class order -- every one with
// even Rc, then every one with odd Rc, index order within each class, each
// class padded to whole tiles -- so p is constant over a tile.  Per (query,
// tile) a lane holds 16 rows of one query column: a v_min3 tree gives the
// tile minimum of Y (about 0.5 VALU op per pair) and one v_lshl_or plus one
// v_min keep the key (Y << b) | tile over a segment of 2^b tiles (b = 11 to 8
// as the widest Y grows with the patch); at each segment's end the key folds
// into the query's (Y, tile) minimum, an earlier segment keeping a tie.  Over
// both lane groups the lexicographic (Y, tile) minimum is in the tile holding
// the (SSD, index) minimum: a row with smaller SSD would have a smaller Y, or
// the same Y and p = 0 (an even-class tile, hence an earlier one); a row with
// the same SSD and a lower index sits in the same class, in the same or an
// earlier tile.  The wavefront then recomputes the exact SSDs of that tile's
// rows in the lane group(s) that reached the minimum and takes their (SSD,
// index) minimum; these gathers overlap the matrix work of the other
// wavefronts on the SIMD.  A launch with at most half as many query chunks
// as resident block slots splits each chunk's reference range over up to
// four blocks, so a small frame fills the chip; the parts leave records that
// a resolve kernel merges before the same check.  Larger launches run whole
// chunks, a nearly empty last round as paired half-size blocks (row_plan).
#pragma once
#include "riann_internal.h"

#include <algorithm>

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

#ifndef RIANN_ROWS_WAVES
#define RIANN_ROWS_WAVES 0                     // 0: four
#endif
#ifndef RIANN_ROWS_QB
#define RIANN_ROWS_QB 0                        // 0: four
#endif
#ifndef RIANN_ROWS_INFLIGHT
#define RIANN_ROWS_INFLIGHT 0                  // 0: by patch width
#endif

// Block shape: wavefronts per block and 32-query column blocks per
// wavefront (WAVES, QB; 0 = the default of the patch width).  Measured on the
// 720p workload (D = 64, dense step): four column blocks and four wavefronts
// 0.73-0.75 ms; three or five column blocks 0.78-0.80 ms; six 0.73-0.76 ms;
// two 0.84 ms; eight wavefronts per block 0.75-0.83 ms.  The defaults are the
// fastest there; the other shapes are built for the autotuner.
template <int DP, int WAVES = 0, int QB = 0>
struct RowCfg {
    static constexpr int waves = WAVES > 0 ? WAVES : (RIANN_ROWS_WAVES > 0 ? RIANN_ROWS_WAVES : 4);
    static constexpr int qb =
        QB > 0 ? QB : (RIANN_ROWS_QB > 0 ? RIANN_ROWS_QB : (DP <= 192 ? 4 : 2));
    // check passes in flight: the wide patches' rows need the registers
    static constexpr int inflight =
        RIANN_ROWS_INFLIGHT > 0 ? RIANN_ROWS_INFLIGHT : (DP <= 96 ? 2 : 1);
    static constexpr int block = 64 * waves;
    static constexpr int wave_q = 32 * qb;
    static constexpr int block_q = wave_q * waves;
    static_assert(qb >= 2, "the LDS prefetch runs one query block ahead");
};
#ifndef RIANN_ROWS_SCHED
// MFMA/VALU interleave: 2 = each MFMA of a chain followed by a share of the
// minimum tree (1: one MFMA, half the tree, the rest; 0: the compiler's
// order).  Measured: 2 and 1 equal at D = 64, 2 faster by 1.8 % at D = 192;
// 0 slower by 3 % at D = 64.  Raising the wave priority around the MFMA
// issue (RIANN_ROWS_SETPRIO) gained nothing.
#define RIANN_ROWS_SCHED 2
#endif
#ifndef RIANN_ROWS_SETPRIO
#define RIANN_ROWS_SETPRIO 0                   // 1: raise wave priority while issuing MFMAs
#endif
#ifndef RIANN_ROWS_LOOKAHEAD
#define RIANN_ROWS_LOOKAHEAD 1                 // MFMA chains issued ahead of the tree
#endif                                         // (2: within 1 %, 25 more registers)
constexpr int kLookahead = RIANN_ROWS_LOOKAHEAD;
#ifndef RIANN_ROWS_XCD_RANGES
#define RIANN_ROWS_XCD_RANGES 1                // 0: whole chunk = block index
#endif
#ifndef RIANN_ROWS_PAIRS
#define RIANN_ROWS_PAIRS 1                     // 0: the last round's chunks run whole
#endif
#ifndef RIANN_ROWS_PAIR_DIV
#define RIANN_ROWS_PAIR_DIV 8                  // pair a last round of <= slots / this chunks
#endif

template <int KB, int ST, int WAVES>
__device__ __forceinline__ void stage_dma(const int8_t *__restrict__ gf,
                                          const int32_t *__restrict__ gh, int sg, int8_t *lf,
                                          int32_t *lh, int wv, int lane) {
    constexpr int CH = ST * KB;
    const int8_t *src = gf + (int64_t)sg * CH * 1024;
#pragma unroll
    for (int i = 0; i < (CH + WAVES - 1) / WAVES; ++i) {
        const int c = wv + WAVES * i;
        if (c < CH)
            __builtin_amdgcn_global_load_lds((glb_void *)(src + c * 1024 + lane * 16),
                                             (lds_void *)(lf + c * 1024), 16, 0, 0);
    }
    if (wv == WAVES - 1 && lane < ST * 8)
        __builtin_amdgcn_global_load_lds((glb_void *)(gh + (int64_t)sg * ST * kTile + lane * 4),
                                         (lds_void *)lh, 16, 0, 0);
}

__device__ __forceinline__ uint32_t min16(const v16i &a) {
    uint32_t m0 = min(min((uint32_t)a[0], (uint32_t)a[1]), (uint32_t)a[2]);
    uint32_t m1 = min(min((uint32_t)a[3], (uint32_t)a[4]), (uint32_t)a[5]);
    uint32_t m2 = min(min((uint32_t)a[6], (uint32_t)a[7]), (uint32_t)a[8]);
    uint32_t m3 = min(min((uint32_t)a[9], (uint32_t)a[10]), (uint32_t)a[11]);
    uint32_t m4 = min(min((uint32_t)a[12], (uint32_t)a[13]), (uint32_t)a[14]);
    m0 = min(min(m0, m1), m2);
    m3 = min(min(m3, m4), (uint32_t)a[15]);
    return min(m0, m3);
}

template <int DP, int ST, int QB, int KN = 1>
struct RowState {
    static constexpr int KB = DP / 32, TB = row_tile_bits(DP);
    v4i Bq[QB][KB];         // query fragments (MFMA B operand)
    uint32_t key[QB];       // min over the current segment of (Y << TB) | tile
    uint32_t bY[QB], bT[QB];// (Y, tile) minimum of the earlier segments
    uint32_t kl[QB][KN];    // k-NN (KN > 1): the KN smallest keys, ascending

    // fold the segment starting at tile t0 into (bY, bT); an earlier segment
    // keeps a tie (its tiles come first)
    __device__ __forceinline__ void fold(uint32_t t0) {
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const uint32_t y = key[qb] >> TB, t = t0 + (key[qb] & ((1u << TB) - 1u));
            const bool lt = y < bY[qb];
            bY[qb] = lt ? y : bY[qb];
            bT[qb] = lt ? t : bT[qb];
            key[qb] = ~0u;
        }
    }

    // A fragments and accumulator initial values (Hf) of tile u of a stage
    __device__ __forceinline__ void load_tile(const int8_t *lf, const int32_t *lh, int u,
                                              int lane, int grp, v4i (&Af)[KB], v16i &H) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            Af[kb] = *reinterpret_cast<const v4i *>(lf + (u * KB + kb) * 1024 + lane * 16);
        const v4i *hp = reinterpret_cast<const v4i *>(lh + u * kTile + grp * 16);
        const v4i h0 = hp[0], h1 = hp[1], h2 = hp[2], h3 = hp[3];
        H = v16i{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3],
                 h2[0], h2[1], h2[2], h2[3], h3[0], h3[1], h3[2], h3[3]};
    }

    __device__ __forceinline__ void mma(int qb, const v4i (&Af)[KB], const v16i &H, v16i &acc) {
        acc = H;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], Bq[qb][kb], acc, 0, 0, 0);
    }

    __device__ __forceinline__ void track(int qb, const v16i &acc, uint32_t t) {
        const uint32_t x0 = (min16(acc) << TB) | t;
        if constexpr (KN == 1) {
            key[qb] = min(key[qb], x0);
        } else {
            uint32_t x = x0;                      // sorted insertion
#pragma unroll
            for (int i = 0; i < KN; ++i) {
                const uint32_t o = kl[qb][i];
                kl[qb][i] = min(o, x);
                x = max(o, x);
            }
        }
    }

    // NT tiles of one LDS stage (all of them, or one half for a wavefront of
    // a pair), as a sequence of (tile, query block) items:
    // the MFMA chain of item i + LA is issued before the minimum tree of
    // item i, so the tree reads an accumulator whose chain has finished while
    // the later chains run (LA + 1 accumulators, used in turn).  The next
    // tile's LDS operands are read one item before its first chain.
    template <int NT>
    __device__ __forceinline__ void stage(const int8_t *lf, const int32_t *lh, uint32_t t0s,
                                          int lane, int grp) {
        constexpr int LA = kLookahead;
        static_assert(QB >= LA + 1, "the next tile's operands load inside the current tile");
        v4i Af[2][KB];
        v16i H[2];
        v16i acc[LA + 1];
        load_tile(lf, lh, 0, lane, grp, Af[0], H[0]);
#pragma unroll
        for (int j = 0; j < LA; ++j) mma(j, Af[0], H[0], acc[j]);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int cur = u & 1;
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                const int it = u * QB + qb, nx = it + LA;
                if (qb == QB - 1 - LA && u + 1 < NT)
                    load_tile(lf, lh, u + 1, lane, grp, Af[cur ^ 1], H[cur ^ 1]);
                if (RIANN_ROWS_SETPRIO) __builtin_amdgcn_s_setprio(1);
                if (nx < NT * QB)
                    mma(nx % QB, Af[(nx / QB) & 1], H[(nx / QB) & 1], acc[nx % (LA + 1)]);
                if (RIANN_ROWS_SETPRIO) __builtin_amdgcn_s_setprio(0);
                track(qb, acc[it % (LA + 1)], t0s + (uint32_t)u);
                if constexpr (RIANN_ROWS_SCHED == 1) {
                    // one MFMA, then half of the tree, then the chain's other
                    // MFMAs and the rest: the wave keeps issuing VALU work
                    // while each MFMA of the chain executes
                    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, KB - 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
                    __builtin_amdgcn_sched_barrier(0);
                } else if constexpr (RIANN_ROWS_SCHED == 2) {
                    // each MFMA of the chain followed by a share of the tree
                    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x002, (10 + KB - 1) / KB, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
};

// Candidate check of one dense query by a 16-lane group.  rec = {Y,
// tile << 2 | group mask}: lane r takes accumulator row r of the tile in each
// masked lane group -- class-order row 32 tile + 8(r/4) + 4g + r%4 -- forms
// its exact SSD with v_dot4 from the row's bytes, and a 16-lane reduction
// keeps the (SSD, reference index) minimum.  The rows come from the
// fragment table the pass stages (already in each XCD's L2) and their
// {Rc, index} from Rci.  (A separate table holding each (tile, group)'s 16
// rows contiguously read fewer lines but measured no faster once the check
// passes were pipelined, and every XCD fetched it into its L2 as well: 1.2 MB
// more per XCD at 720p.)  issue() starts the loads that need only the record (Qc
// and the first masked group's row with its {Rc, index}); finish() takes the
// query patch (global memory or LDS), Qc and the query's frame and does the
// rest, so a caller can have the loads of several queries in flight before
// any waits.  A record whose group mask is 0 means no check (not live).
template <int DP>
struct RowCheck {
    static constexpr int KB = DP / 32;
    uint4 v[DP / 16];       // first candidate row of this lane (patch byte order)
    int2 ri;                // its {Rc, reference index}; index < 0: none

    __device__ __forceinline__ static void row_bytes(const DevIndex &ix, int64_t tile, int m,
                                                     uint4 (&v)[DP / 16]) {
        // fragment order: tile, k-block kb, lane m + 32h -> bytes 32kb + 16h of row m
        const uint4 *f = reinterpret_cast<const uint4 *>(ix.Rfr) + tile * KB * 64 + m;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            v[2 * kb] = f[kb * 64];
            v[2 * kb + 1] = f[kb * 64 + 32];
        }
    }

    // accumulator row r of lane group g of a tile (tile row 8(r/4) + 4g +
    // r%4) and its {Rc, index}
    __device__ __forceinline__ static void check_row(const DevIndex &ix, int64_t tile, int g, int r,
                                                     uint4 (&v)[DP / 16], int2 &ci) {
        const int m = 8 * (r >> 2) + 4 * g + (r & 3);
        row_bytes(ix, tile, m, v);
        ci = ix.Rci[tile * kTile + m];
    }

    // (the loads are unconditional -- a record without a group reads a row of
    // tile 0 and drops it -- so a pass's loads stay countable in flight)
    __device__ __forceinline__ void issue(const DevIndex &ix, const uint2 &rec, int r) {
        const int g = (rec.y & 1u) ? 0 : 1;
        check_row(ix, rec.y >> 2, g, r, v, ri);
        if ((rec.y & 3u) == 0u) ri = make_int2(0, -1);
    }

    __device__ __forceinline__ static int dot(const uint4 (&a)[DP / 16], const uint4 (&v)[DP / 16]) {
        int d = 0;
#pragma unroll
        for (int k = 0; k < DP / 16; ++k) {
            d = __builtin_amdgcn_sdot4((int)a[k].x, (int)v[k].x, d, false);
            d = __builtin_amdgcn_sdot4((int)a[k].y, (int)v[k].y, d, false);
            d = __builtin_amdgcn_sdot4((int)a[k].z, (int)v[k].z, d, false);
            d = __builtin_amdgcn_sdot4((int)a[k].w, (int)v[k].w, d, false);
        }
        return d;
    }

    // min over the 16 lanes of a DPP row (one query's group): quad swaps,
    // then the mirrored half-row and row, each lane ending with the minimum
    template <int CTRL>
    __device__ __forceinline__ static unsigned long long dpp_min(unsigned long long b) {
        const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
        const unsigned hi =
            (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        return o < b ? o : b;
    }

    // ONE: a one-frame launch, whose field, SSD map and first query the
    // caller passes as uniform values (out0, ssd0, qb0); otherwise the
    // query's frame fid selects them from the descriptor table
    template <bool ONE>
    __device__ __forceinline__ void finish(const DevIndex &ix, const FrameBatch &fb, uint32_t q,
                                           const uint2 &rec, int qc, int fid, int lane,
                                           const uint4 *patch, int32_t *out0, uint32_t *ssd0,
                                           int64_t qb0) {
        const int r = lane & 15;
        const bool live = (rec.y & 3u) != 0u;
        unsigned long long best = ~0ull;
        if (live) {
            uint4 a[DP / 16];
#pragma unroll
            for (int k = 0; k < DP / 16; ++k) a[k] = patch[k];
            if (ri.y >= 0) {
                const uint32_t ssd = (uint32_t)(qc + ri.x + 2 * dot(a, v));
                best = ((unsigned long long)ssd << 32) | (uint32_t)ri.y;
            }
            if ((rec.y & 3u) == 3u) {           // both lane groups reached the minimum
                uint4 u[DP / 16];
                int2 rj;
                check_row(ix, rec.y >> 2, 1, r, u, rj);
                if (rj.y >= 0) {
                    const uint32_t ssd = (uint32_t)(qc + rj.x + 2 * dot(a, u));
                    const unsigned long long k2 = ((unsigned long long)ssd << 32) | (uint32_t)rj.y;
                    best = k2 < best ? k2 : best;
                }
            }
        }
        best = dpp_min<0xB1>(best);             // quad_perm [1,0,3,2]
        best = dpp_min<0x4E>(best);             // quad_perm [2,3,0,1]
        best = dpp_min<0x141>(best);            // row_half_mirror
        best = dpp_min<0x140>(best);            // row_mirror
        if (live && r == 0) {
            int32_t *out = out0;
            uint32_t *ssd = ssd0;
            int64_t qbase = qb0;
            if constexpr (!ONE) {
                const FrameDesc *fdp = &fb.f[fid];
                out = fdp->out;
                ssd = fdp->ssd;
                qbase = fdp->qbase;
            }
            const int64_t ql = (int64_t)q - qbase;
            out[ql] = (int32_t)(uint32_t)best;
            if (ssd) ssd[ql] = (uint32_t)(best >> 32);
        }
    }
};

// The candidate checks of a wavefront's 32 QB queries after its pass over
// the references: 8 QB passes of four queries (one per 16-lane group), each
// pass's candidate rows requested IF - 1 passes ahead, so a pass waits only
// on its own loads.  The records, query ids, Qc and frame ids come from the
// owning lanes by shuffles; the patches from LDS (STAGED) or global memory.
template <int DP, int QB, int IF, bool STAGED, bool ONE>
__device__ __forceinline__ void check_wave(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                           const uint2 (&rc)[QB], const uint32_t (&qid)[QB],
                                           const int (&qcl)[QB], const int (&fidl)[QB],
                                           const int8_t *sp, int lane) {
    constexpr int NP = QB * 8;
    const int sub = lane >> 4, r = lane & 15;
    int32_t *out0 = nullptr;
    uint32_t *ssd0 = nullptr;
    int64_t qb0 = 0;
    if constexpr (ONE) {
        out0 = fb.f[0].out;
        ssd0 = fb.f[0].ssd;
        qb0 = fb.f[0].qbase;
    }
    RowCheck<DP> C[IF];
    uint2 rr[IF];
    uint32_t qq[IF];
    int qc[IF], fd[IF];
    auto fetch = [&](int k) {
        const int s = k % IF, qb = k / 8, c = (k % 8) * 4 + sub;
        rr[s] = make_uint2(__shfl(rc[qb].x, c, 64), __shfl(rc[qb].y, c, 64));
        qq[s] = (uint32_t)__shfl((int)qid[qb], c, 64);
        qc[s] = __shfl(qcl[qb], c, 64);
        fd[s] = ONE ? 0 : __shfl(fidl[qb], c, 64);
        C[s].issue(ix, rr[s], r);
    };
#pragma unroll
    for (int k = 0; k < IF - 1 && k < NP; ++k) fetch(k);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (k + IF - 1 < NP) fetch(k + IF - 1);
        const int s = k % IF, qb = k / 8, c = (k % 8) * 4 + sub;
        const int8_t *patch = STAGED ? sp + (qb * 32 + c) * DP
                                     : reinterpret_cast<const int8_t *>(w.patches) +
                                           (int64_t)qq[s] * DP;
        C[s].template finish<ONE>(ix, fb, qq[s], rr[s], qc[s], fd[s], lane,
                                  reinterpret_cast<const uint4 *>(patch), out0, ssd0, qb0);
    }
}

// How a launch covers `chunks` query chunks with `slots` resident blocks:
// the first `whole` chunks run as one block each over every reference; each
// later chunk is split over `parts` blocks (consecutive blocks, consecutive
// parts).  Only a launch with at most half as many chunks as slots splits:
// every chunk into as many parts as fit the slots in one round (at most
// kRowMaxParts), so a small frame still fills the chip.  A larger launch runs
// whole chunks only, except that when its last round holds at most an
// eighth of the slots its `paired` chunks each run as two blocks of half the
// queries, the wavefronts of each block in two halves over the same queries,
// each half over half of every stage's tiles, merging their minima in LDS (no
// records, no resolve pass): those few blocks, alone on their CUs, then end
// about twice as soon.  Measured at D = 64 with 768 slots: a last round of 32
// or 96 chunks -7 % and -6 % of the launch; 160 and 192 unchanged; 237 (a
// 720p frame) +0.7 %; 384 -2 %.  (Splitting the last round over reference
// parts instead measured no faster: each part re-read its chunk's patches and
// the resolve pass re-read records and candidate rows.)  Blocks used: whole +
// 2 paired, or whole + (chunks - whole) * parts <= chunks + min(3 * chunks,
// slots).
struct RowPlan {
    uint32_t whole, parts, paired;
};
__host__ __device__ inline RowPlan row_plan(uint32_t chunks, uint32_t slots, bool pair_ok) {
    const uint32_t cap = (uint32_t)kRowMaxParts;
    if (chunks == 0 || slots == 0) return RowPlan{chunks, 1u, 0u};
    if (chunks > slots) {
        const uint32_t tail = chunks % slots;
        const uint32_t pr = pair_ok && tail <= slots / RIANN_ROWS_PAIR_DIV ? tail : 0u;
        return RowPlan{chunks - pr, 1u, pr};
    }
    uint32_t p = slots / chunks;
    p = p < cap ? p : cap;
    return p > 1 ? RowPlan{0u, p, 0u} : RowPlan{chunks, 1u, 0u};
}

// Bytes [o, o + 8) of the frame as two words: the aligned words holding
// them, realigned (the third only when o is not word-aligned: every word read
// holds a byte of the frame).
__device__ __forceinline__ uint2 frame_bytes8(const uint8_t *p) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const uint32_t r = (uint32_t)(a & 3u);
    const uint32_t *d = reinterpret_cast<const uint32_t *>(a - r);
    const uint32_t d0 = d[0], d1 = d[1];
    const uint32_t d2 = r ? d[2] : 0u;
    return make_uint2(__builtin_amdgcn_alignbyte(d1, d0, r), __builtin_amdgcn_alignbyte(d2, d1, r));
}

// The fused dense search's own patch assembly (8 x 8 gray, one frame): query
// q's MFMA B fragments -- bytes 32 kb + 16 grp .. + 16 of the patch in
// (dy, dx) order, rows 4 kb + 2 grp and the next, encoded a = q ^ 0x7F --
// and its Qc = sum (a + 1)^2 over the 64 bytes, the lane pair (grp 0 and 1)
// each summing its half.  The extraction kernel's encoding, done in place.
__device__ __forceinline__ void fused_patch(const FrameDesc &fa, int s, uint32_t q, int grp,
                                            v4i (&Bq)[2], int &qc) {
    const uint32_t qy = q / (uint32_t)fa.Wq, qx = q - qy * (uint32_t)fa.Wq;
    const uint8_t *base = fa.frame + (int64_t)qy * s * fa.pitch + (int64_t)qx * s;
    int sa2 = 0, sa = 0;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const int dy = 4 * kb + 2 * grp;
        const uint2 r0 = frame_bytes8(base + (int64_t)dy * fa.pitch);
        const uint2 r1 = frame_bytes8(base + (int64_t)(dy + 1) * fa.pitch);
        const uint32_t wd[4] = {r0.x ^ 0x7F7F7F7Fu, r0.y ^ 0x7F7F7F7Fu, r1.x ^ 0x7F7F7F7Fu,
                                r1.y ^ 0x7F7F7F7Fu};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sa2 = __builtin_amdgcn_sdot4((int)wd[i], (int)wd[i], sa2, false);
            sa = __builtin_amdgcn_sdot4((int)wd[i], 0x01010101, sa, false);
        }
        Bq[kb] = v4i{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3]};
    }
    sa2 += __shfl_xor(sa2, 32, 64);
    sa += __shfl_xor(sa, 32, 64);
    qc = sa2 + 2 * sa + 64;
}

// A fused ring frame's routing counts, as the extraction kernel would have
// made them: every query goes dense, those with a valid previous match on
// the bound m* >= 1, the others as no-prior queries (m* = n).  Lane group 0
// of each wavefront counts its 32 QB queries; pv holds their previous
// matches, read before the pass over the references.
template <int QB>
__device__ __forceinline__ void fused_counts(const DevIndex &ix, const FrameBatch &fb,
                                             uint32_t wbase, uint32_t count,
                                             const int32_t (&pv)[QB], int lane) {
    unsigned long long nq = 0, np = 0;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const bool valid = lane < 32 && wbase + (uint32_t)(qb * 32 + lane) < count;
        const bool noprior = pv[qb] < 0 || (int64_t)pv[qb] >= ix.n;
        nq += (unsigned long long)__popcll(__ballot(valid));
        np += (unsigned long long)__popcll(__ballot(valid && noprior));
    }
    if (lane == 0 && nq) {
        stat_add(fb.stats, ST_QUERIES, nq);
        stat_add(fb.stats, ST_DENSE, nq);
        if (np) {
            stat_add(fb.stats, ST_NOPRIOR, np);
            stat_add(fb.stats, ST_MSTAR, np * (unsigned long long)ix.n);
        }
        if (nq > np) stat_add(fb.stats, ST_BOUND, nq - np);
    }
}

template <int DP, int ST, int WAVES = 0, int QB = 0>
__global__ __launch_bounds__((RowCfg<DP, WAVES, QB>::block)) void k_dense_rows(DevIndex ix,
                                                                            FrameBatch fb, Work w,
                                                                            uint32_t slots) {
    using Cfg = RowCfg<DP, WAVES, QB>;
    constexpr int KB = DP / 32;
    constexpr int kWaves = Cfg::waves, kQB = Cfg::qb;
    constexpr int kWaveQ = Cfg::wave_q, kBlockQ = Cfg::block_q;
    constexpr int STAGE = ST * KB * 1024;
    // the two reference stages; after the last tile, the query patches of
    // narrow patches (wide ones are read from global memory by the check)
    constexpr bool kStagePatches = DP <= 96;
    // each stage buffer is its own LDS array, so the compiler can tell a
    // read of one from the DMA filling the other and need not wait for the
    // DMA before computing on the first; after the last tile the two hold
    // the query patches, the first half of the wavefronts' in each
    constexpr int HALF_PATCHES = kStagePatches ? kBlockQ * DP / 2 : 0;
    constexpr int HALF = STAGE > HALF_PATCHES ? STAGE : HALF_PATCHES;
    constexpr int SPS = (1 << row_tile_bits(DP)) / ST;  // stages per key segment
    static_assert(SPS % 2 == 0, "stage pairs never straddle a segment");
    static_assert(kWaves % 2 == 0, "the patch staging splits the wavefronts in halves");
    // paired chunks need an even split of the tiles and of the query blocks
    constexpr int kHalfW = kWaves / 2, kHalfQB = kQB / 2;
    constexpr bool kPair = RIANN_ROWS_PAIRS && ST % 2 == 0 && kQB % 2 == 0;
    static_assert(kWaves * kQB * 64 * 8 <= HALF, "the pair exchange fits one stage buffer");
    __shared__ __attribute__((aligned(16))) int8_t s_f0[HALF];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[HALF];
    __shared__ __attribute__((aligned(16))) int32_t s_h0[ST * kTile];
    __shared__ __attribute__((aligned(16))) int32_t s_h1[ST * kTile];

    // the queries in order (a full search, or a ring launch whose route codes
    // mark the ring-scanned ones), or the dense list
    const bool natural = fb.all_full || fb.dense_masked;
    const uint32_t *list = natural ? nullptr : w.dense_list;
    const uint32_t count = natural ? (uint32_t)fb.Q : w.counters[1];
    // whole chunks first, then the split ones, nsplit blocks per chunk, each
    // over one part of the reference stages (consecutive blocks take
    // consecutive parts and land on different XCDs, so each XCD's L2 holds
    // fewer parts)
    const RowPlan plan = row_plan((count + kBlockQ - 1) / kBlockQ, slots, kPair);
    const uint32_t bx = blockIdx.x;
    const bool whole = bx < plan.whole;
    // a half of a paired chunk (after the whole chunks; plan.parts is 1)
    const bool paired = kPair && !whole && plan.paired > 0;
    const int nsplit = whole || paired ? 1 : (int)plan.parts;
    const uint32_t split = whole || paired ? 0u : (bx - plan.whole) % plan.parts;
    // whole chunks by XCD bands: each XCD's L2 then holds the frame rows of
    // one contiguous range of queries instead of rows from all of them
    const uint32_t wc = RIANN_ROWS_XCD_RANGES && whole ? xcd_band(bx, plan.whole) : bx;
    const uint32_t chunk = whole ? wc : paired ? bx : plan.whole + (bx - plan.whole) / plan.parts;
    const uint32_t qbase = paired ? plan.whole * kBlockQ + (bx - plan.whole) * (kBlockQ / 2)
                                  : chunk * kBlockQ;
    const uint32_t nbq = paired ? kBlockQ / 2 : kBlockQ;   // the block's queries
    if (qbase >= count) return;                   // whole block exits together
    if (fb.dense_masked == kDenseMasked) {
        // a chunk whose queries the ring scan answers, all of them, has no work
        bool any = false;
        for (uint32_t i = threadIdx.x; i < nbq; i += Cfg::block)
            any = any || (qbase + i < count && w.route[qbase + i] != kRouteScan);
        if (!__syncthreads_or(any)) return;
    }

    // the wavefront index is uniform: keep it (and the DMA addresses) in SGPRs
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31, grp = lane >> 5;
    // in a paired block, wavefronts wq and wq + kHalfW hold the same queries,
    // the first over tiles [0, ST / 2) of every stage, the second over the rest
    const int half = paired ? wv / kHalfW : 0;
    const int wq = paired ? wv % kHalfW : wv;
    const int ns_all = (int)(ix.n_rows / (kTile * ST));
    const int s_begin = (int)((int64_t)split * ns_all / nsplit);
    const int s_end = (int)((int64_t)(split + 1) * ns_all / nsplit);

    if (s_begin < s_end) stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, s_begin, s_f0, s_h0, wv, lane);

    RowState<DP, ST, kQB> S;
    uint32_t qid[kQB];
    int qcf[kQB];                                 // Qc of this lane's queries (fused)
    const bool fused = DP == 64 && fb.fused;
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wq * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        qcf[qb] = 0;
        bool built = false;
        if constexpr (DP == 64) {
            if (fused) {
                fused_patch(fb.f[0], ix.s, qid[qb], grp, S.Bq[qb], qcf[qb]);
                built = true;
            }
        }
        if (!built) {
            const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) +
                                (int64_t)qid[qb] * DP + grp * 16;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                S.Bq[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
        }
        S.key[qb] = ~0u;
        S.bY[qb] = ~0u;
        S.bT[qb] = 0u;
    }
    // a fused ring frame's previous matches, counted after the pass (one
    // part of a split chunk counts its queries)
    const bool counts = fused && !fb.all_full && split == 0 && half == 0;
    int32_t pvq[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb)
        pvq[qb] = counts && grp == 0 && fb.f[0].prev ? fb.f[0].prev[qid[qb]] : -1;
    __syncthreads();

    // one stage's tiles: all of them, or this wavefront's half in a pair
    auto run_stage = [&](const int8_t *lf, const int32_t *lh, uint32_t t0s) {
        if constexpr (kPair) {
            if (paired) {
                constexpr int NH = ST / 2;
                S.template stage<NH>(lf + half * (NH * KB * 1024), lh + half * (NH * kTile),
                                     t0s + (uint32_t)(half * NH), lane, grp);
                return;
            }
        }
        S.template stage<ST>(lf, lh, t0s, lane, grp);
    };
    int seg0 = s_begin;                           // first stage of the key segment
    for (int sg = s_begin; sg < s_end; sg += 2) {
        if (sg - seg0 == SPS) {
            S.fold((uint32_t)(seg0 * ST));
            seg0 = sg;
        }
        if (sg + 1 < s_end) stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, sg + 1, s_f1, s_h1, wv, lane);
        run_stage(s_f0, s_h0, (uint32_t)((sg - seg0) * ST));
        __syncthreads();
        if (sg + 1 < s_end) {
            if (sg + 2 < s_end) stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, sg + 2, s_f0, s_h0, wv, lane);
            run_stage(s_f1, s_h1, (uint32_t)((sg + 1 - seg0) * ST));
            __syncthreads();
        }
    }
    S.fold((uint32_t)(seg0 * ST));
    if (counts) fused_counts(ix, fb, qbase + (uint32_t)(wq * kWaveQ), count, pvq, lane);
    if constexpr (kPair) {
        if (paired) {
            // the two wavefronts of a pair saw disjoint tiles of the same
            // queries: each takes the lexicographic (Y, tile) minimum of both,
            // exchanged through a stage buffer (no DMA is in flight here)
            uint2 *xo = reinterpret_cast<uint2 *>(s_f0) + wv * (kQB * 64);
            const uint2 *xi =
                reinterpret_cast<const uint2 *>(s_f0) + ((wv + kHalfW) % kWaves) * (kQB * 64);
#pragma unroll
            for (int qb = 0; qb < kQB; ++qb) xo[qb * 64 + lane] = make_uint2(S.bY[qb], S.bT[qb]);
            __syncthreads();
#pragma unroll
            for (int qb = 0; qb < kQB; ++qb) {
                const uint2 o = xi[qb * 64 + lane];
                const bool lt = o.x < S.bY[qb] || (o.x == S.bY[qb] && o.y < S.bT[qb]);
                S.bY[qb] = lt ? o.x : S.bY[qb];
                S.bT[qb] = lt ? o.y : S.bT[qb];
            }
        }
    }

    // ---- merge the two lane groups (rows 0-15 and 16-31 of every tile's
    // accumulator order): the lexicographically smaller (Y, tile) wins; equal
    // pairs mean the same Y in the same tile, checked in both groups.
    // rec = {Y, tile << 2 | group mask}, the tile counted over the whole class
    // order, the same in both groups.
    uint2 rc[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t y = S.bY[qb], t = S.bT[qb];
        const uint32_t oy = (uint32_t)__shfl_xor((int)y, 32, 64);
        const uint32_t ot = (uint32_t)__shfl_xor((int)t, 32, 64);
        const bool same = y == oy && t == ot;
        const bool mine = y < oy || (y == oy && t < ot);
        const uint32_t gm = same ? 3u : (mine ? (1u << grp) : (2u >> grp));
        rc[qb] = make_uint2(mine || same ? y : oy, ((mine || same ? t : ot) << 2) | gm);
    }

    const uint32_t wbase = qbase + (uint32_t)(wq * kWaveQ);
    if (nsplit > 1) {
        // one part of the reference range: the record goes to the resolve
        // kernel at the query's dense-list position (the records are free
        // once the ring scan has run)
        uint4 *dst = split ? w.rec2 + (int64_t)(split - 1) * w.capacity : w.rec;
#pragma unroll
        for (int qb = 0; qb < kQB; ++qb) {
            const uint32_t slot = wbase + (uint32_t)(qb * 32 + col);
            if (slot < count && grp == 0) dst[slot] = make_uint4(rc[qb].x, rc[qb].y, 0u, 0u);
            if (fused && split == 0 && slot < count) {
                // the resolve pass checks these queries from their stored
                // patches and Qc, which no extraction kernel wrote
                int8_t *pd = reinterpret_cast<int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                             grp * 16;
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    *reinterpret_cast<v4i *>(pd + kb * 32) = S.Bq[qb][kb];
                if (grp == 0) w.qc[qid[qb]] = qcf[qb];
            }
        }
        return;
    }
    // the whole reference range: the wavefront checks its own queries
    // (check_wave), the query patches from the MFMA operand registers
    // through the (now free) stage buffers.
    int8_t *const sp = (wv < kWaves / 2 ? s_f0 : s_f1) + (wv % (kWaves / 2)) * (kWaveQ * DP);
    if constexpr (kStagePatches) {
        __syncthreads();                          // every wavefront is past its last tile
#pragma unroll
        for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                *reinterpret_cast<v4i *>(sp + (qb * 32 + col) * DP + kb * 32 + grp * 16) =
                    S.Bq[qb][kb];
        __syncthreads();
    }
    // each lane's own queries: Qc, frame id and liveness (past the dense
    // count, or answered by the ring scan: group mask 0) read once, all
    // loads together and unconditionally (every array holds the launch's
    // queries), before the passes
    int qcl[kQB], fidl[kQB];
    uint32_t code[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        if (fused) {                              // one frame, every query dense
            qcl[qb] = qcf[qb];
            fidl[qb] = 0;
            code[qb] = kRouteFull;
        } else {
            qcl[qb] = w.qc[qid[qb]];              // qid is a valid query (clamped slot)
            fidl[qb] = (int)w.fid[qid[qb]];
            code[qb] = w.route[qid[qb]];
        }
    }
    const uint32_t masked = fb.dense_masked == kDenseMasked ? 1u : 0u;
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t in = wbase + (uint32_t)(qb * 32 + col) < count ? 1u : 0u;
        const uint32_t scan = code[qb] == (uint32_t)kRouteScan ? 1u : 0u;
        rc[qb].y = (in & (masked & scan ^ 1u)) ? rc[qb].y : 0u;
    }
    if constexpr (kPair) {
        if (paired) {
            // the two wavefronts of a pair hold the same merged records:
            // each checks half of the query blocks
            uint2 rh[kHalfQB];
            uint32_t qh[kHalfQB];
            int ch[kHalfQB], fh[kHalfQB];
#pragma unroll
            for (int i = 0; i < kHalfQB; ++i) {
                const int j = i + kHalfQB;
                rh[i] = half ? rc[j] : rc[i];
                qh[i] = half ? qid[j] : qid[i];
                ch[i] = half ? qcl[j] : qcl[i];
                fh[i] = half ? fidl[j] : fidl[i];
            }
            const int8_t *sph = sp + half * (kHalfQB * 32 * DP);
            if (fb.n == 1)
                check_wave<DP, kHalfQB, Cfg::inflight, kStagePatches, true>(ix, fb, w, rh, qh, ch,
                                                                           fh, sph, lane);
            else
                check_wave<DP, kHalfQB, Cfg::inflight, kStagePatches, false>(ix, fb, w, rh, qh, ch,
                                                                            fh, sph, lane);
            return;
        }
    }
    if (fb.n == 1)
        check_wave<DP, kQB, Cfg::inflight, kStagePatches, true>(ix, fb, w, rc, qid, qcl, fidl, sp,
                                                               lane);
    else
        check_wave<DP, kQB, Cfg::inflight, kStagePatches, false>(ix, fb, w, rc, qid, qcl, fidl, sp,
                                                                lane);
}

template <int DP, int BQ>
__global__ __launch_bounds__(256) void k_resolve(DevIndex ix, FrameBatch fb, Work w, uint32_t slots) {
    constexpr uint32_t kBlockQ = BQ;                 // queries per chunk of the row kernel
    const bool natural = fb.all_full || fb.dense_masked;
    const uint32_t *list = natural ? nullptr : w.dense_list;
    const uint32_t count = natural ? (uint32_t)fb.Q : w.counters[1];
    const RowPlan plan = row_plan((count + kBlockQ - 1) / kBlockQ, slots, false);
    const int nsplit = (int)plan.parts;
    const int lane = threadIdx.x & 63, r = lane & 15;
    for (uint32_t base = plan.whole * kBlockQ + blockIdx.x * 16u; base < count;
         base += gridDim.x * 16u) {
        const uint32_t i = base + (threadIdx.x >> 4);
        const bool live = i < count &&
                          (fb.dense_masked != kDenseMasked || w.route[i] != kRouteScan);
        const uint32_t q = live ? (list ? list[i] : i) : 0u;
        uint2 rec = make_uint2(0u, 0u);
        if (live) {
            unsigned long long best = ~0ull;
#pragma unroll
            for (int s = 0; s < kRowMaxParts; ++s) {
                if (s < nsplit) {
                    const uint4 p = s ? w.rec2[(int64_t)(s - 1) * w.capacity + i] : w.rec[i];
                    const unsigned long long k = ((unsigned long long)p.x << 32) | p.y;
                    best = k < best ? k : best;
                }
            }
            rec = make_uint2((uint32_t)(best >> 32), (uint32_t)best);
        }
        const int qc = live ? w.qc[q] : 0;
        const int fid = live && fb.n > 1 ? (int)w.fid[q] : 0;
        RowCheck<DP> C;
        C.issue(ix, rec, r);
        C.template finish<false>(ix, fb, q, rec, qc, fid, lane,
                                 reinterpret_cast<const uint4 *>(w.patches + (int64_t)q * DP),
                                 nullptr, nullptr, 0);
    }
}

template <int DP, int WAVES = 0, int QB = 0>
hipError_t launch_rows_t(const DevIndex &ix, const FrameBatch &fb, const Work &w, hipStream_t st) {
    using Cfg = RowCfg<DP, WAVES, QB>;
    constexpr int ST = DP <= 64 ? 8 : 4;
    static_assert(kRowAlign % (kTile * ST) == 0, "reference padding must cover whole stages");
    // The dense query count is known on the device only: the grid covers the
    // largest plan any count up to fb.Q can take, and surplus blocks return
    // at once.  (Splitting every chunk of a 720p frame -- 1,773 chunks on
    // 768 slots -- costs more than it gains: the query patches are read once
    // per part and every query goes through the resolve kernel.)
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(&k_dense_rows<DP, ST, WAVES, QB>), Cfg::block, 0);
        resident = std::max(1, cus) * std::max(1, per);
    }
    constexpr int kBlockQ = Cfg::block_q;
    const int64_t chunks = std::max<int64_t>(1, (fb.Q + kBlockQ - 1) / kBlockQ);
    const uint32_t slots = (uint32_t)resident;
    const int64_t blocks = chunks + std::min<int64_t>(3 * chunks, resident);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense_rows<DP, ST, WAVES, QB>), dim3((unsigned)blocks),
                       dim3(Cfg::block), 0, st, ix, fb, w, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // split queries: fewer than min(chunks, slots) chunks' worth.  With the
    // queries in order the plan is known here: no split, no resolve pass
    if ((fb.all_full || fb.dense_masked) &&
        row_plan((uint32_t)std::min<int64_t>(chunks, 0x7FFFFFFF), slots, false).parts == 1)
        return hipSuccess;
    const int64_t sq = std::min<int64_t>(chunks, resident) * kBlockQ;
    const int64_t rb = std::min<int64_t>((sq + 15) / 16, 4096);   // 16 queries per 256-thread block
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_resolve<DP, kBlockQ>), dim3((unsigned)rb), dim3(256),
                       0, st, ix, fb, w, slots);
    return hipGetLastError();
}

}  // namespace

}  // namespace riann
