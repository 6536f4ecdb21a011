// k_dense_rows.hip -- exact exhaustive search with references as the MFMA
// rows and queries as the columns (v_mfma_i32_32x32x32_i8), for narrow
// patches (Dp <= 96) where the column layout is bound by its epilogue.
//
// With a = 127 - q, v = r - 128 and p = Rc & 1, the per-reference value
// Hf = (Rc + bias - p) / 2 enters as the MFMA's C operand, read straight from
// LDS, so the accumulator is Y = Hf + <a, v> and SSD - Qc + bias = 2Y + p
// exactly.  Per (query, tile) a lane holds 16 rows of one query column: a
// v_min3 tree gives the tile minimum of Y (about 0.5 VALU op per pair) and a
// few compares keep, per query, the smallest Y and the first tile attaining
// it.  After its last tile the wavefront recomputes the exact SSDs of that
// tile's rows in the lane group(s) that reached the minimum and takes their
// (SSD, index) minimum -- the global one, because every row elsewhere has a
// larger Y, hence a larger SSD (2Y + p grows with Y); these gathers overlap
// the matrix work of the other wavefronts on the SIMD.  The smallest Y can
// occur in several tiles (references whose SSDs differ by one share a Y), so
// each lane also keeps the latest later tile with an equal minimum and a
// count of them; the check then covers up to two tiles, and the rare query
// whose minimum Y sits in three or more tiles is answered by an exhaustive
// per-query search (fallback list).  For small frames the reference range is
// split over up to four blocks per query chunk; the parts then leave records
// that a resolve kernel merges before the same check.
#include "riann_internal.h"

#include <algorithm>

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

#ifndef RIANN_ROWS_WAVES
#define RIANN_ROWS_WAVES 4
#endif
#ifndef RIANN_ROWS_QB
#define RIANN_ROWS_QB 4
#endif
constexpr int kWaves = RIANN_ROWS_WAVES;
constexpr int kBlock = 64 * kWaves;
constexpr int kQB = RIANN_ROWS_QB;     // 32-query column blocks per wavefront
static_assert(kQB >= 2, "the LDS prefetch runs one query block ahead");
constexpr int kWaveQ = 32 * kQB;
constexpr int kBlockQ = kWaveQ * kWaves;
constexpr int kMaxSplit = 4;                   // reference-range parts per query chunk
#ifndef RIANN_ROWS_SPLIT
#define RIANN_ROWS_SPLIT 0                     // 0: chosen per launch
#endif

template <int KB, int ST>
__device__ __forceinline__ void stage_dma(const int8_t *__restrict__ gf,
                                          const int32_t *__restrict__ gh, int sg, int8_t *lf,
                                          int32_t *lh, int wv, int lane) {
    constexpr int CH = ST * KB;
    const int8_t *src = gf + (int64_t)sg * CH * 1024;
#pragma unroll
    for (int i = 0; i < (CH + kWaves - 1) / kWaves; ++i) {
        const int c = wv + kWaves * i;
        if (c < CH)
            __builtin_amdgcn_global_load_lds((glb_void *)(src + c * 1024 + lane * 16),
                                             (lds_void *)(lf + c * 1024), 16, 0, 0);
    }
    if (wv == kWaves - 1 && lane < ST * 8)
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

template <int DP, int ST>
struct RowState {
    static constexpr int KB = DP / 32;
    v4i Bq[kQB][KB];        // query fragments (MFMA B operand)
    uint32_t bY[kQB];       // smallest Y so far (this lane's 16 rows)
    uint32_t bT[kQB];       // first tile attaining it
    uint32_t bT2[kQB];      // the latest later tile reaching the same Y
    uint32_t cnt[kQB];      // how many later tiles reached it

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
        const uint32_t m = min16(acc);
        const bool lt = m < bY[qb];
        const bool eq = m == bY[qb];
        bT2[qb] = eq ? t : bT2[qb];
        cnt[qb] = lt ? 0u : cnt[qb] + (eq ? 1u : 0u);
        bT[qb] = lt ? t : bT[qb];
        bY[qb] = lt ? m : bY[qb];
    }

    // all tiles of one LDS stage; the MFMA chain of the next query block (or
    // of the next tile's first block) is issued before the current block's
    // minimum tree, so the matrix core and the VALU overlap.  The next tile's
    // LDS operands are read one query block ahead.
    __device__ __forceinline__ void stage(const int8_t *lf, const int32_t *lh, uint32_t t0s,
                                          int lane, int grp) {
        v4i Af[2][KB];
        v16i H[2];
        v16i acc[2];
        load_tile(lf, lh, 0, lane, grp, Af[0], H[0]);
        mma(0, Af[0], H[0], acc[0]);
#pragma unroll
        for (int u = 0; u < ST; ++u) {
            const int cur = u & 1;
#pragma unroll
            for (int qb = 0; qb < kQB; ++qb) {
                if (qb == kQB - 2 && u + 1 < ST)
                    load_tile(lf, lh, u + 1, lane, grp, Af[cur ^ 1], H[cur ^ 1]);
                if (qb + 1 < kQB)
                    mma(qb + 1, Af[cur], H[cur], acc[(qb + 1) & 1]);
                else if (u + 1 < ST)
                    mma(0, Af[cur ^ 1], H[cur ^ 1], acc[0]);
                track(qb, acc[qb & 1], t0s + (uint32_t)u);
                // one MFMA, then half of the tree, then the chain's second
                // MFMA and the rest: the wave keeps issuing VALU work while
                // each MFMA of the chain executes
                __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, KB - 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
};

// Candidate check of one dense query by a 16-lane group: lane r takes
// accumulator row r of each recorded (tile, lane group) -- tile row
// 8(r/4) + 4g + r%4 -- forms its exact SSD with v_dot4, and a 16-lane
// reduction keeps the (SSD, index) minimum, which is the global one since
// every other row has a larger Y.  rec = {Y, T1 << 2 | group mask, T2 + 1
// (0: none), fallback}.  load() issues the query patch and the first
// candidate row, finish() does the rest, so a caller can issue the loads of
// two queries before either waits.  Queries flagged for the fallback are
// appended to the fallback list and counted; finish() is called by every lane
// of the wavefront (the append is a wave-wide ballot).
template <int DP>
struct RowCheck {
    uint4 a[DP / 16];       // query patch
    uint4 v[DP / 16];       // first candidate row of this lane
    int64_t ref0;           // its index (-1: none)
    int qc;

    __device__ __forceinline__ void load(const DevIndex &ix, const Work &w, uint32_t q,
                                         const uint4 &rec, bool live, int r) {
        ref0 = -1;
        if (!live || rec.w) return;
        const uint4 *src = reinterpret_cast<const uint4 *>(w.patches + (int64_t)q * DP);
#pragma unroll
        for (int k = 0; k < DP / 16; ++k) a[k] = src[k];
        qc = w.qc[q];
        // the first candidate is always tile T1, in the first masked group
        const int g = (rec.y & 1u) ? 0 : 1;
        const int64_t ref = (int64_t)(rec.y >> 2) * kTile + 8 * (r >> 2) + 4 * g + (r & 3);
        if (ref < ix.n) {
            ref0 = ref;
            const uint4 *row = reinterpret_cast<const uint4 *>(ix.Rv + ref * DP);
#pragma unroll
            for (int k = 0; k < DP / 16; ++k) v[k] = row[k];
        }
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

    __device__ __forceinline__ void finish(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                           unsigned long long *stats, uint32_t q,
                                           const uint4 &rec, bool live, int lane) {
        const int r = lane & 15;
        const bool fbk = rec.w != 0;
        unsigned long long best = ~0ull;
        if (live && !fbk) {
            if (ref0 >= 0) {
                const uint32_t ssd = (uint32_t)(qc + ix.Rc[ref0] + 2 * dot(a, v));
                best = ((unsigned long long)ssd << 32) | (uint32_t)ref0;
            }
            // the other candidates: the second group of T1, then T2 (rare)
            const uint32_t gm = rec.y & 3u;
            const uint32_t tiles[2] = {rec.y >> 2, rec.z - 1};
            const int ntl = rec.z ? 2 : 1;
            const int c0 = (gm & 1u) ? 0 : 1;
#pragma unroll
            for (int c = 1; c < 4; ++c) {
                const int tt = c >> 1, g = c & 1;
                const int64_t ref = (int64_t)tiles[tt] * kTile + 8 * (r >> 2) + 4 * g + (r & 3);
                if (c > c0 && tt < ntl && ((gm >> g) & 1u) && ref < ix.n) {
                    uint4 u[DP / 16];
                    const uint4 *row = reinterpret_cast<const uint4 *>(ix.Rv + ref * DP);
#pragma unroll
                    for (int k = 0; k < DP / 16; ++k) u[k] = row[k];
                    const uint32_t ssd = (uint32_t)(qc + ix.Rc[ref] + 2 * dot(a, u));
                    const unsigned long long key = ((unsigned long long)ssd << 32) | (uint32_t)ref;
                    best = key < best ? key : best;
                }
            }
        }
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) {
            const unsigned lo = __shfl_xor((unsigned)best, m, 64);
            const unsigned hi = __shfl_xor((unsigned)(best >> 32), m, 64);
            const unsigned long long o = ((unsigned long long)hi << 32) | lo;
            best = o < best ? o : best;
        }
        if (live && !fbk && r == 0) {
            const FrameDesc *fdp = &fb.f[w.fid[q]];
            const int64_t ql = (int64_t)q - fdp->qbase;
            fdp->out[ql] = (int32_t)(uint32_t)best;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(best >> 32);
        }
        const bool mine = live && fbk && r == 0;
        const unsigned long long fmask = __ballot(mine);
        if (fmask) {
            uint32_t base = 0;
            if (lane == 0) {
                base = atomicAdd(&w.counters[2], (uint32_t)__popcll(fmask));
                atomicAdd(&stats[ST_FALLBACK], (unsigned long long)__popcll(fmask));
            }
            base = __shfl(base, 0, 64);
            if (mine) {
                const unsigned lo = __builtin_amdgcn_mbcnt_lo((unsigned)fmask, 0u);
                w.fb_list[base + __builtin_amdgcn_mbcnt_hi((unsigned)(fmask >> 32), lo)] = q;
            }
        }
    }
};

template <int DP, int ST>
__global__ __launch_bounds__(kBlock) void k_dense_rows(DevIndex ix, FrameBatch fb, Work w,
                                                       unsigned long long *stats, int nsplit) {
    constexpr int KB = DP / 32;
    constexpr int STAGE = ST * KB * 1024;
    __shared__ __attribute__((aligned(16))) int8_t s_f0[STAGE];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[STAGE];
    __shared__ __attribute__((aligned(16))) int32_t s_h0[ST * kTile];
    __shared__ __attribute__((aligned(16))) int32_t s_h1[ST * kTile];

    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t count = fb.all_full ? (uint32_t)fb.Q : w.counters[1];
    // nsplit blocks per query chunk, each over one part of the reference
    // stages (consecutive blocks take consecutive parts and land on
    // different XCDs, so each XCD's L2 holds fewer parts)
    const uint32_t split = blockIdx.x % (uint32_t)nsplit;
    const uint32_t qbase = (blockIdx.x / (uint32_t)nsplit) * kBlockQ;
    if (qbase >= count) return;                   // whole block exits together

    // the wavefront index is uniform: keep it (and the DMA addresses) in SGPRs
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31, grp = lane >> 5;
    const int ns_all = (int)(ix.n_pad / (kTile * ST));
    const int s_begin = (int)((int64_t)split * ns_all / nsplit);
    const int s_end = (int)((int64_t)(split + 1) * ns_all / nsplit);

    if (s_begin < s_end) stage_dma<KB, ST>(ix.Rf, ix.Hf, s_begin, s_f0, s_h0, wv, lane);

    RowState<DP, ST> S;
    uint32_t qid[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                            grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) S.Bq[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
        S.bY[qb] = ~0u;
        S.bT[qb] = 0;
        S.bT2[qb] = 0;
        S.cnt[qb] = 0;
    }
    __syncthreads();

    for (int sg = s_begin; sg < s_end; sg += 2) {
        if (sg + 1 < s_end) stage_dma<KB, ST>(ix.Rf, ix.Hf, sg + 1, s_f1, s_h1, wv, lane);
        S.stage(s_f0, s_h0, (uint32_t)(sg * ST), lane, grp);
        __syncthreads();
        if (sg + 1 < s_end) {
            if (sg + 2 < s_end) stage_dma<KB, ST>(ix.Rf, ix.Hf, sg + 2, s_f0, s_h0, wv, lane);
            S.stage(s_f1, s_h1, (uint32_t)((sg + 1) * ST), lane, grp);
            __syncthreads();
        }
    }

    // ---- merge the two lane groups (rows 0-15 and 16-31 of every tile's
    // accumulator order) into one record per query, the same in both groups:
    // rec = {Y, T1 << 2 | group mask, T2 + 1 (0: none), fallback}.  The
    // minimum Y sits in tile T1 (and T2) within the masked groups' rows;
    // three or more tiles go to the fallback.
    uint4 rc[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t y = S.bY[qb], t = S.bT[qb], t2 = S.bT2[qb], c = S.cnt[qb];
        const uint32_t oY = (uint32_t)__shfl_xor((int)y, 32, 64);
        const uint32_t oT = (uint32_t)__shfl_xor((int)t, 32, 64);
        const uint32_t oT2 = (uint32_t)__shfl_xor((int)t2, 32, 64);
        const uint32_t oC = (uint32_t)__shfl_xor((int)c, 32, 64);
        uint32_t T1, T2p = 0, gm, fbk = 0;
        if (y != oY) {
            const bool own = y < oY;
            const uint32_t cc = own ? c : oC;
            T1 = own ? t : oT;
            gm = own ? (1u << grp) : (2u >> grp);
            if (cc == 1) T2p = (own ? t2 : oT2) + 1;
            if (cc > 1) fbk = 1;
        } else if (c > 1 || oC > 1) {
            T1 = min(t, oT); gm = 3u; fbk = 1;
        } else {
            // distinct tiles among t (< t2) and oT (< oT2)
            const uint32_t a1 = t, a2 = c ? t2 : t, b1 = oT, b2 = oC ? oT2 : oT;
            const uint32_t lo = min(a1, b1);
            uint32_t hi = lo, n = 1;
            const uint32_t cand[4] = {a1, a2, b1, b2};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (cand[k] != lo && (n == 1 || cand[k] != hi)) {
                    if (n == 1) { hi = cand[k]; n = 2; } else { n = 3; }
                }
            }
            T1 = lo; gm = 3u;
            if (n == 2) T2p = hi + 1;
            if (n > 2) fbk = 1;
        }
        rc[qb] = make_uint4(min(y, oY), (T1 << 2) | gm, T2p, fbk);
    }

    const uint32_t wbase = qbase + (uint32_t)(wv * kWaveQ);
    if (nsplit > 1) {
        // one part of the reference range: the record goes to the resolve
        // kernel at the query's dense-list position (the records are free
        // once the ring scan has run)
        uint4 *dst = split ? w.rec2 + (int64_t)(split - 1) * w.capacity : w.rec;
#pragma unroll
        for (int qb = 0; qb < kQB; ++qb) {
            const uint32_t slot = wbase + (uint32_t)(qb * 32 + col);
            if (slot < count && grp == 0) dst[slot] = rc[qb];
        }
        return;
    }
    // the whole reference range: the wavefront checks its own queries, four
    // at a time (one per 16-lane group), the loads of two such passes in
    // flight together; the records and query ids come from the owning lanes
    const int sub = lane >> 4, r = lane & 15;
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        for (int h = 0; h < 32; h += 8) {
            const int ca = h + sub, cb = h + 4 + sub;
            const uint4 ra = make_uint4(__shfl(rc[qb].x, ca, 64), __shfl(rc[qb].y, ca, 64),
                                        __shfl(rc[qb].z, ca, 64), __shfl(rc[qb].w, ca, 64));
            const uint4 rb = make_uint4(__shfl(rc[qb].x, cb, 64), __shfl(rc[qb].y, cb, 64),
                                        __shfl(rc[qb].z, cb, 64), __shfl(rc[qb].w, cb, 64));
            const uint32_t qa = (uint32_t)__shfl((int)qid[qb], ca, 64);
            const uint32_t qbq = (uint32_t)__shfl((int)qid[qb], cb, 64);
            const bool la = wbase + (uint32_t)(qb * 32 + ca) < count;
            const bool lb = wbase + (uint32_t)(qb * 32 + cb) < count;
            RowCheck<DP> A, B;
            A.load(ix, w, qa, ra, la, r);
            B.load(ix, w, qbq, rb, lb, r);
            A.finish(ix, fb, w, stats, qa, ra, la, lane);
            B.finish(ix, fb, w, stats, qbq, rb, lb, lane);
        }
    }
}

// Resolve step of a launch whose reference range is split over several
// blocks per query chunk: 16 lanes per dense query merge the parts' records
// (the smallest Y wins; parts that tie on it contribute their tiles, disjoint
// ranges, checked in both lane groups -- more than two tiles in all go to the
// fallback) and run the candidate check.  The records sit at the list
// position, so they load alongside the list.
template <int DP>
__global__ __launch_bounds__(256) void k_resolve(DevIndex ix, FrameBatch fb, Work w,
                                                 unsigned long long *stats, int nsplit) {
    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t count = fb.all_full ? (uint32_t)fb.Q : w.counters[1];
    const int lane = threadIdx.x & 63, r = lane & 15;
    const uint32_t i = blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = i < count;
    const uint32_t q = live ? (list ? list[i] : i) : 0u;
    uint4 rec = make_uint4(0u, 0u, 0u, 1u);
    if (live) {
        uint4 rp[kMaxSplit];
        uint32_t ymin = ~0u;
#pragma unroll
        for (int s = 0; s < kMaxSplit; ++s) {
            if (s < nsplit) {
                rp[s] = s ? w.rec2[(int64_t)(s - 1) * w.capacity + i] : w.rec[i];
                ymin = min(ymin, rp[s].x);
            }
        }
        uint32_t t[2] = {0u, 0u}, gm = 0u, fb = 0u;
        int nt = 0, nrec = 0;
#pragma unroll
        for (int s = 0; s < kMaxSplit; ++s) {
            if (s < nsplit && rp[s].x == ymin) {
                ++nrec;
                fb |= rp[s].w;
                gm |= rp[s].y & 3u;
                if (nt < 2) t[nt] = rp[s].y >> 2;
                ++nt;
                if (rp[s].z) {
                    if (nt < 2) t[nt] = rp[s].z - 1;
                    ++nt;
                }
            }
        }
        // one record keeps its own group mask; tiles from several records are
        // checked in both groups
        if (nrec > 1) gm = 3u;
        rec = make_uint4(ymin, (t[0] << 2) | gm, nt > 1 ? t[1] + 1 : 0u,
                         (fb || nt > 2) ? 1u : 0u);
    }
    RowCheck<DP> C;
    C.load(ix, w, q, rec, live, r);
    C.finish(ix, fb, w, stats, q, rec, live, lane);
}

// Exhaustive exact search for the few queries of a list: one block per query
// (grid-stride over the list, whose length is read on the device), each of
// its 1024 threads takes every 1024th reference with v_dot4, and a block
// reduction keeps the (SSD, index) minimum.  Every block leaves the loop once
// its index passes the count.
constexpr int kBruteT = 1024;

template <int DP>
__global__ __launch_bounds__(kBruteT) void k_brute_list(DevIndex ix, FrameBatch fb, Work w,
                                                    const uint32_t *__restrict__ list,
                                                    const uint32_t *__restrict__ count_ptr) {
    __shared__ unsigned long long s_red[kBruteT / 64];
    const uint32_t count = *count_ptr;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const uint32_t q = list[i];
        uint32_t a[DP / 4];
        const uint4 *src = reinterpret_cast<const uint4 *>(w.patches + (int64_t)q * DP);
#pragma unroll
        for (int k = 0; k < DP / 16; ++k) {
            const uint4 v = src[k];
            a[4 * k] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
        }
        const int Qc = w.qc[q];
        unsigned long long best = ~0ull;
        for (int64_t r = tid; r < ix.n; r += kBruteT) {
            const uint4 *row = reinterpret_cast<const uint4 *>(ix.Rv + r * DP);
            int d = 0;
#pragma unroll
            for (int k = 0; k < DP / 16; ++k) {
                const uint4 v = row[k];
                d = __builtin_amdgcn_sdot4((int)a[4 * k], (int)v.x, d, false);
                d = __builtin_amdgcn_sdot4((int)a[4 * k + 1], (int)v.y, d, false);
                d = __builtin_amdgcn_sdot4((int)a[4 * k + 2], (int)v.z, d, false);
                d = __builtin_amdgcn_sdot4((int)a[4 * k + 3], (int)v.w, d, false);
            }
            const uint32_t ssd = (uint32_t)(Qc + ix.Rc[r] + 2 * d);
            const unsigned long long key = ((unsigned long long)ssd << 32) | (uint32_t)r;
            best = key < best ? key : best;
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const unsigned lo = __shfl_xor((unsigned)best, m, 64);
            const unsigned hi = __shfl_xor((unsigned)(best >> 32), m, 64);
            const unsigned long long o = ((unsigned long long)hi << 32) | lo;
            best = o < best ? o : best;
        }
        if (lane == 0) s_red[wv] = best;
        __syncthreads();
        if (tid == 0) {
            unsigned long long b = s_red[0];
            for (int k = 1; k < kBruteT / 64; ++k) b = s_red[k] < b ? s_red[k] : b;
            const FrameDesc *fdp = &fb.f[w.fid[q]];
            const int64_t ql = (int64_t)q - fdp->qbase;
            fdp->out[ql] = (int32_t)(uint32_t)b;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(b >> 32);
        }
        __syncthreads();
    }
}

template <int DP>
hipError_t launch_rows_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                         unsigned long long *stats, hipStream_t st) {
    constexpr int ST = DP <= 64 ? 8 : 4;
    static_assert(kRefAlign % (kTile * ST) == 0, "reference padding must cover whole stages");
    // Split the reference range over nsplit blocks per query chunk only when
    // there are too few chunks to give every resident block slot one (small
    // frames); measured on a 720p frame (1,773 chunks, 768 slots) splitting
    // costs more -- the query patches are read once per part -- than its
    // shorter last round gains.
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void *>(&k_dense_rows<DP, ST>), kBlock, 0);
        resident = std::max(1, cus) * std::max(1, per);
    }
    const int64_t chunks = std::max<int64_t>(1, (fb.Q + kBlockQ - 1) / kBlockQ);
    int nsplit = (int)std::min<int64_t>(kMaxSplit, (resident + chunks - 1) / chunks);
#if RIANN_ROWS_SPLIT > 0
    nsplit = RIANN_ROWS_SPLIT;
#endif
    const int64_t blocks = nsplit * chunks;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense_rows<DP, ST>), dim3((unsigned)blocks), dim3(kBlock),
                       0, st, ix, fb, w, stats, nsplit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nsplit > 1) {
        // the parts meet in a resolve step (one part: the row kernel checks
        // its own candidates)
        const int64_t rb = (fb.Q + 15) / 16;      // 16 queries per 256-thread block
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_resolve<DP>), dim3((unsigned)(rb < 1 ? 1 : rb)),
                           dim3(256), 0, st, ix, fb, w, stats, nsplit);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the fallback list is short; at most 256 blocks walk it
    const int64_t fbl = fb.Q < 256 ? (fb.Q < 1 ? 1 : fb.Q) : 256;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_brute_list<DP>), dim3((unsigned)fbl), dim3(kBruteT), 0, st,
                       ix, fb, w, (const uint32_t *)w.fb_list, (const uint32_t *)(w.counters + 2));
    return hipGetLastError();
}

}  // namespace

bool dense_rows_supported(const DevIndex &ix) { return ix.Dp <= 96; }

hipError_t launch_dense_rows(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             unsigned long long *stats, hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_rows_t<32>(ix, fb, w, stats, st);
    case 64: return launch_rows_t<64>(ix, fb, w, stats, st);
    case 96: return launch_rows_t<96>(ix, fb, w, stats, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
