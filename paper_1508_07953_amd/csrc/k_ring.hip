// k_ring.hip -- ring phase and ring scan of the exact-mode RIANN search.
//
// k_ring (one lane per query) follows the per-query steps of Algorithm 1:
//   extract q; c = SSD(q, R[prev]) (radius^2 from the previous match);
//   b_k = SSD(q, key_k); ring k = [lo_k, hi_k] in key-distance space with
//   integer bounds (no rounding slack); a lower and an upper position bound
//   in key k's sorted list give [st_k, en_k) (Sec. 3.3: a ring costs two
//   binary searches); the smallest ring k* is kept; the query is routed to
//   the ring scan when m* = en - st is small and to the dense search
//   otherwise.  Per-key bucket counts bound every m_k first, so the binary
//   searches run only for the keys that can still hold the smallest ring.
// k_scan (one wavefront per routed query) scans key k*'s ring, keeps the
//   references inside all K rings (the intersection S) and takes the argmin
//   of the exact SSD over S with a wavefront reduction (lowest index on ties).
#include "riann_internal.h"
#include "ring_math.h"

#include <algorithm>

namespace riann {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl_xor(lo, m, 64);
    hi = __shfl_xor(hi, m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += shfl_xor_u64(v, m);
    return v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        unsigned long long o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t isqrt_u64(uint64_t x) {
    uint64_t s = (uint64_t)sqrt((double)x);
    while (s * s > x) --s;
    while ((s + 1) * (s + 1) <= x) ++s;
    return s;
}

// Integer ring of one key: references r with |sqrt(a) - sqrt(b)| <= sqrt(c),
// a = SSD(r, key), b = SSD(q, key): lo <= a <= hi.
__device__ __forceinline__ void ring_bounds(uint32_t b, uint32_t c, uint32_t &lo, uint32_t &hi) {
    uint64_t s = isqrt_u64(4ull * b * c);
    lo = (b <= c) ? 0u : (uint32_t)((uint64_t)b + c - s);
    hi = (uint32_t)((uint64_t)b + c + s);
}

// Positions in a key's sorted list: the number of entries with x < v
// (LE = false, the lower_bound of v) or x <= v (LE = true, the upper_bound).
// sample_count searches the list's samples (S[i] = T[16 s0l i], ns of them,
// a table that stays in L2) and returns how many satisfy the predicate; that brackets the
// position (pos_bracket).  exact_pos finishes the search in global memory:
// a binary search over the first entries of 16-entry lines, then one
// aligned 64-byte line is read and counted.
template <bool LE>
__device__ __forceinline__ bool pred(uint32_t x, uint32_t v) { return LE ? x <= v : x < v; }

template <bool LE>
__device__ __forceinline__ int sample_count(const uint32_t *S, int ns, uint32_t v,
                                            uint32_t &probes) {
    int lo = 0, len = ns;
    while (len > 0) {
        const int half = len >> 1;
        ++probes;
        if (pred<LE>(S[lo + half], v)) { lo += half + 1; len -= half + 1; }
        else len = half;
    }
    return lo;
}

// position range [pl, ph] implied by the sample count i
__device__ __forceinline__ void pos_bracket(int i, int ns, int s0l, uint32_t n, uint32_t &pl,
                                            uint32_t &ph) {
    if (i == 0) { pl = ph = 0; return; }
    pl = 16u * (uint32_t)((i - 1) * s0l) + 1u;
    ph = i < ns ? min(16u * (uint32_t)(i * s0l), n) : n;
}

template <bool LE>
__device__ __forceinline__ uint32_t exact_pos(int i, const uint32_t *__restrict__ T, int nlines,
                                              int s0l, uint32_t v, uint32_t &probes) {
    if (i == 0) return 0;
    int L = (i - 1) * s0l, H = min(i * s0l, nlines);
    while (H - L > 1) {
        const int mid = (L + H) >> 1;
        ++probes;
        if (pred<LE>(T[16 * mid], v)) L = mid;
        else H = mid;
    }
    ++probes;                                  // the 64-byte line read below
    const uint4 *line = reinterpret_cast<const uint4 *>(T + 16 * L);
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 x = line[q];
        cnt += pred<LE>(x.x, v) + pred<LE>(x.y, v) + pred<LE>(x.z, v) + pred<LE>(x.w, v);
    }
    return 16u * (uint32_t)L + cnt;
}

// b = SSD(q, key k) from the key rows staged in LDS (k rows of Dp bytes,
// then the keys' Rc).
template <int DP>
__device__ __forceinline__ uint32_t key_dist(const uint32_t (&a)[DP / 4], int Qc,
                                             const uint32_t *krows, const uint32_t *krc, int k) {
    const int d = dot_row<DP>(a, reinterpret_cast<const int8_t *>(krows + k * (DP / 4)));
    return (uint32_t)(Qc + (int)krc[k] + 2 * d);
}

__device__ __forceinline__ uint32_t lane_prefix(unsigned long long mask) {
    unsigned m = __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u);
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), m);
}

// ---------------------------------------------------------------- k_scan_rows
// The ring scan over the ring-ordered pivot rows (the default layout): entry
// j of key k's sorted list carries its reference's whole pivot row,
// PivR[k][j] = Piv[P[k][j]] (KQ 16-byte words per row, padding keys 0), so
// the smallest ring [st, en) of key k* is one contiguous stream of rows that
// consecutive lanes read from consecutive addresses.  Each lane keeps U rows
// in flight.  Ring k's test lo_k <= x <= hi_k is the unsigned
// x - lo_k <= hi_k - lo_k; padding keys get [0, 2^32 - 1], which every
// value meets.  The reference index (P) is read only for candidates inside
// every ring, before their exact SSD.  One wavefront scans one query (rec =
// {c, k*, st, en}) and writes its match; returns |S| (on every lane).
template <int DP, int KQ, int U>
__device__ __forceinline__ uint32_t scan_query(const DevIndex &ix, const FrameBatch &fb,
                                               const Work &w, uint32_t qid, const uint4 rec,
                                               int lane) {
    const uint32_t n = (uint32_t)ix.n;
    const uint32_t c = rec.x, ks = rec.y, st = rec.z, en = rec.w;
    const uint32_t mine = lane < DP / 4
        ? reinterpret_cast<const uint32_t *>(w.patches + (int64_t)qid * DP)[lane] : 0u;
    uint32_t a[DP / 4];
#pragma unroll
    for (int i = 0; i < DP / 4; ++i) a[i] = (uint32_t)__builtin_amdgcn_readlane((int)mine, i);
    const int Qc = w.qc[qid];
    uint32_t lo = 0, wd = 0xFFFFFFFFu;
    if (lane < ix.K) {
        const int key = ix.keys[lane];
        const int d = dot_row<DP>(a, ix.Rv + (int64_t)key * ix.Dp);
        const uint32_t b = (uint32_t)(Qc + ix.Rc[key] + 2 * d);
        uint32_t hi;
        ring_bounds(b, c, lo, hi);
        wd = hi - lo;
    }
    unsigned long long best = ~0ull;
    uint32_t cnt = 0;
    const int32_t *Pk = ix.P + (int64_t)ks * n;
    const uint4 *rows = reinterpret_cast<const uint4 *>(ix.PivR) + (int64_t)ks * ix.n16 * KQ;
    for (uint32_t j0 = st; j0 < en; j0 += 64 * U) {
        uint4 pv[U][KQ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + 64 * u + lane;
            const uint4 *row = rows + (int64_t)(j < en ? j : st) * KQ;
#pragma unroll
            for (int q = 0; q < KQ; ++q) pv[u][q] = row[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + 64 * u + lane;
            bool in = j < en;
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const uint32_t x[4] = {pv[u][q].x, pv[u][q].y, pv[u][q].z, pv[u][q].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)lo, 4 * q + e);
                    const uint32_t wk = (uint32_t)__builtin_amdgcn_readlane((int)wd, 4 * q + e);
                    in = in && x[e] - lk <= wk;
                }
            }
            if (in) {
                ++cnt;
                const int32_t r = Pk[j];
                const int d = dot_row<DP>(a, ix.Rv + (int64_t)r * ix.Dp);
                const uint32_t s = (uint32_t)(Qc + ix.Rc[r] + 2 * d);
                const unsigned long long key = ((unsigned long long)s << 32) | (uint32_t)r;
                best = key < best ? key : best;
            }
        }
    }
    best = wave_min_u64(best);
    const uint32_t tot = (uint32_t)wave_sum_u64(cnt);
    if (lane == 0) {
        const FrameDesc *fdp = &fb.f[w.fid[qid]];
        const int64_t ql = (int64_t)qid - fdp->qbase;
        fdp->out[ql] = (int32_t)(uint32_t)best;
        if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(best >> 32);
    }
    return tot;
}

// One wavefront per item of the ring list (grid-stride).
template <int DP, int KQ>
__global__ __launch_bounds__(kBlock) void k_scan_rows(DevIndex ix, FrameBatch fb, Work w,
                                                       unsigned long long *__restrict__ stats) {
    constexpr int U = KQ <= 4 ? 4 : (KQ <= 8 ? 2 : 1);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t count = w.counters[0];
    unsigned long long surv_tot = 0, mstar_tot = 0;
    for (uint32_t item = blockIdx.x * (kBlock / 64) + wv; item < count;
         item += gridDim.x * (kBlock / 64)) {
        const uint32_t qid = w.ring_list[item];
        const uint4 rec = w.rec[qid];
        const uint32_t tot = scan_query<DP, KQ, U>(ix, fb, w, qid, rec, lane);
        if (lane == 0) {
            surv_tot += tot;
            mstar_tot += rec.w - rec.z;
        }
    }
    __shared__ unsigned long long s_acc[kBlock / 64][2];
    if (lane == 0) { s_acc[wv][0] = surv_tot; s_acc[wv][1] = mstar_tot; }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long tot = 0;
        for (int i = 0; i < kBlock / 64; ++i) tot += s_acc[i][threadIdx.x];
        if (tot) stat_add(stats, threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING, tot);
    }
}

// ---------------------------------------------------------------- k_ring
// One lane per query.  The extraction kernel before it has already sent
// full-search queries, queries without a prior and queries whose every ring
// certainly exceeds the routing threshold to the dense search (route codes):
// this kernel only appends those to the dense list and counts them.  A block
// with any other query first copies into LDS each key's bucket-count row and
// the key rows with their Rc.  Then, per remaining query:
//  1. every key's ring-size bounds [lb_k, ub_k] from its bucket counts, with
//     an inner and an outer fp32 approximation of the ring (no exact square
//     root yet); the seed key is the smallest lb (lowest k on ties).  If
//     that lb is above the routing threshold, every ring holds more than the
//     threshold's candidates: the query goes to the dense list with no exact
//     ring (unless the index asks for every query's exact m*);
//  2. the seed's exact ring: exact bounds, the samples bracket the two
//     positions, two line reads in global memory fix them;
//  3. the remaining keys whose lower bound can still beat (m, k) -- chosen
//     against the seed's exact size when the bounds stay in registers (K <= 16,
//     Dp <= 64), else against the smallest upper bound -- each lane taking
//     its own keys in turn; a key is searched only while (lb, k) and then its
//     sample bracket (ml, k) are below the best (m, k), and wins on a smaller
//     size or an equal one at a lower index.
// The result -- the exact smallest ring m*, its key k* (lowest on ties) and
// its range -- is the same as evaluating every key exactly; the routing
// decision (m* <= threshold) is the same with or without step 1's shortcut.
// List appends and statistics are aggregated per block: one atomic per list
// and per counter per block.
// Queries per block: 1024, or 512 for the variant that keeps the bounds of
// up to 16 keys in registers (80 VGPRs: six wavefronts per SIMD fit in three
// 512-query blocks, not in 1024-query ones).
__host__ __device__ constexpr int ring_block(int KR) { return KR > 0 ? 512 : 1024; }

template <int DP, int KR, int KQ>
__global__ __launch_bounds__(ring_block(KR), KR > 0 ? 6 : 1) void k_ring(DevIndex ix, FrameBatch fb, Work w,
                                                      unsigned long long *__restrict__ stats,
                                                      int64_t threshold) {
    constexpr int kBlk = ring_block(KR), kWv = kBlk / 64;
    extern __shared__ __attribute__((aligned(16))) uint32_t s_samp[];
    __shared__ uint32_t s_wcnt[kWv][2];
    __shared__ uint32_t s_base[2];
    __shared__ unsigned long long s_st[kWv][6];
    // KQ > 0: the block scans its own ring queries (ring-ordered pivot rows
    // of KQ 16-byte words), listed here, instead of the ring list
    __shared__ uint32_t s_rq[KQ > 0 ? kBlk : 1];
    __shared__ uint4 s_rr[KQ > 0 ? kBlk : 1];
    __shared__ unsigned long long s_sc[KQ > 0 ? kWv : 1][2];
    const int64_t Q = fb.Q;
    // (blocks in XCD bands, as the dense search takes its chunks, measured
    // 2-4 % slower here: a band of costly rings loads one XCD)
    const uint32_t bx = blockIdx.x;
    const int64_t qid = (int64_t)bx * kBlk + threadIdx.x;
    const bool valid = qid < Q;
    const int64_t qq = valid ? qid : Q - 1;
    // the extraction kernel has already routed full-search, no-prior and
    // bound-routed queries (route codes); the rest need this kernel's work.
    // With fb.dense_masked the extraction kernel has also counted the routed
    // ones, so a block with no other query has nothing to do; otherwise it
    // still appends them to the dense list and counts them, without staging
    const uint8_t code = w.route[qq];
    const bool work = valid && code == kRouteRing;
    const bool any_work = __syncthreads_or(work);
    if (fb.dense_masked && !any_work) return;
    // queries whose statistics this kernel counts
    const bool counted = fb.dense_masked ? work : valid;
    // LDS: the bucket-count rows, then the key rows and their Rc (the binary
    // searches' samples are read from L2, where the whole table stays)
    constexpr int olb = 0;
    const int olk = olb + ix.K * ix.lbS;
    const int olc = olk + ix.K * (DP / 4);
    if (any_work) {
        for (int i = threadIdx.x; i < ix.K * ix.lbS / 4; i += kBlk)
            reinterpret_cast<uint4 *>(s_samp + olb)[i] = reinterpret_cast<const uint4 *>(ix.Lb)[i];
        for (int i = threadIdx.x; i < ix.K * (DP / 16); i += kBlk) {
            const int k = i / (DP / 16), part = i - k * (DP / 16);
            reinterpret_cast<uint4 *>(s_samp + olk)[i] =
                reinterpret_cast<const uint4 *>(ix.Rv + (int64_t)ix.keys[k] * ix.Dp)[part];
        }
        for (int k = threadIdx.x; k < ix.K; k += kBlk) s_samp[olc + k] = (uint32_t)ix.Rc[ix.keys[k]];
        __syncthreads();
    }

    const uint32_t n = (uint32_t)ix.n;
    const int nlines = ix.n16 / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const FrameDesc *fdp = &fb.f[w.fid[qq]];
    const bool full = fdp->mode == kModeFull;
    const int32_t *prev = full ? nullptr : fdp->prev;
    const int64_t ql = qq - fdp->qbase;
    uint32_t a[DP / 4] = {};
    int Qc = 0;
    if (work) {
        const uint4 *src = reinterpret_cast<const uint4 *>(w.patches + qq * DP);
#pragma unroll
        for (int i = 0; i < DP / 16; ++i) {
            const uint4 v = src[i];
            a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
        }
        Qc = w.qc[qq];
    }
    // radius: the SSD to the previous match; for k-NN fields the largest SSD
    // to the k previous matches, which must be k distinct references (then
    // the k nearest lie within it); anything else means no prior
    bool noprior = prev == nullptr || code == kRouteNoPrior;
    uint32_t c = 0xFFFFFFFFu;
    if (work && !noprior) {
        const int kn = fb.knn;
        uint32_t cm = 0;
        for (int j = 0; j < kn && !noprior; ++j) {
            const int32_t pv = prev[ql * kn + j];
            if (pv < 0 || (int64_t)pv >= ix.n) { noprior = true; break; }
            for (int j2 = 0; j2 < j; ++j2)
                if (prev[ql * kn + j2] == pv) noprior = true;
            int d = dot_row<DP>(a, ix.Rv + (int64_t)pv * ix.Dp);
            cm = max(cm, (uint32_t)(Qc + ix.Rc[pv] + 2 * d));
        }
        if (!noprior) c = cm;
    }
    uint32_t best_m = n, best_k = 0, best_st = 0, best_en = n;
    uint32_t probes = 0;                      // sorted-table reads of the binary searches
    // routed by the extraction kernel on the same ring-size bounds: every
    // ring holds more than the threshold's candidates
    bool by_bound = code == kRouteBound;
    if (work && !full && !noprior && ix.K > 0) {
        const uint32_t *LB = s_samp + olb, *KR_ = s_samp + olk, *KC = s_samp + olc;
        const int B = ix.lbB, LS = ix.lbS;
        // 1. every key's ring-size bounds from its bucket counts: the seed is
        //    the smallest lower bound (lowest key on ties); keys whose lower
        //    bound exceeds the smallest upper bound so far cannot hold the
        //    smallest ring, the others are marked (a superset of the keys
        //    the exact search below may need)
        uint32_t k1 = 0, lb1 = 0xFFFFFFFFu, b1 = 0, ubmin = 0xFFFFFFFFu;
        unsigned long long cand = 0;
        uint32_t lbv[KR > 0 ? KR : 1];            // KR > 0: every key's lower bound
        auto bound_key = [&](int k) {
            const uint32_t b = key_dist<DP>(a, Qc, KR_, KC, k);
            uint32_t li, hi_, lo_, ho;
            ring_approx(b, c, li, hi_, lo_, ho);
            uint32_t lb, ub;
            ring_size_bounds(LB + k * LS, B, li, hi_, lo_, ho, lb, ub);
            ubmin = min(ubmin, ub);
            if (lb < lb1) { lb1 = lb; k1 = (uint32_t)k; b1 = b; }
            return lb;
        };
        if constexpr (KR > 0) {
            // all K <= KR keys unrolled, so the bounds stay in registers and
            // the candidates are chosen against the seed's exact size below
#pragma unroll
            for (int k = 0; k < KR; ++k) lbv[k] = k < ix.K ? bound_key(k) : 0xFFFFFFFFu;
        } else {
            for (int k = 0; k < ix.K; ++k) {
                const uint32_t lb = bound_key(k);
                if (lb <= ubmin) cand |= 1ull << k;
            }
        }
        // every ring holds more than the threshold's candidates: the query
        // goes dense whatever its exact m* (unless every m* is asked for)
        by_bound = !ix.exact_mstar && (int64_t)lb1 > threshold;
        if (by_bound) {
            best_m = lb1;
            best_k = k1;
        } else {
            // 2. the seed's exact ring
            {
                uint32_t lo1, hi1;
                ring_bounds(b1, c, lo1, hi1);
                const uint32_t *S = ix.Ts + (int64_t)k1 * ix.ns;
                const int il = sample_count<false>(S, ix.ns, lo1, probes);
                const int ih = sample_count<true>(S, ix.ns, hi1, probes);
                const uint32_t *t = ix.T + (int64_t)k1 * ix.n16;
                best_st = exact_pos<false>(il, t, nlines, ix.s0l, lo1, probes);
                best_en = exact_pos<true>(ih, t, nlines, ix.s0l, hi1, probes);
                best_m = best_en - best_st;
                best_k = k1;
            }
            if constexpr (KR > 0) {
                // keys whose lower bound can still beat (best_m, best_k)
#pragma unroll
                for (int k = 0; k < KR; ++k)
                    if (lbv[k] < best_m || (lbv[k] == best_m && (uint32_t)k < best_k))
                        cand |= 1ull << k;
            }
            cand &= ~(1ull << k1);
            // 3. each lane takes its own remaining keys in turn (the wavefront
            //    loops as often as its busiest lane needs): a key is searched
            //    only if its bounds can still beat (best_m, best_k), and wins on
            //    a smaller size or an equal size at a lower index
            while (__ballot(cand != 0)) {
                if (cand == 0) continue;
                const int k = __builtin_ctzll(cand);
                cand &= cand - 1;
                uint32_t lo, hi;
                ring_bounds(key_dist<DP>(a, Qc, KR_, KC, k), c, lo, hi);
                uint32_t lb, ub;
                ring_size_bounds(LB + k * LS, B, lo, hi, lo, hi, lb, ub);
                if (lb > best_m || (lb == best_m && (uint32_t)k > best_k)) continue;
                const uint32_t *S = ix.Ts + (int64_t)k * ix.ns;
                const int il = sample_count<false>(S, ix.ns, lo, probes);
                const int ih = sample_count<true>(S, ix.ns, hi, probes);
                uint32_t sl, sh, el, eh;
                pos_bracket(il, ix.ns, ix.s0l, n, sl, sh);
                pos_bracket(ih, ix.ns, ix.s0l, n, el, eh);
                const uint32_t ml = el > sh ? el - sh : 0u;
                if (ml > best_m || (ml == best_m && (uint32_t)k > best_k)) continue;
                const uint32_t *t = ix.T + (int64_t)k * ix.n16;
                const uint32_t st = exact_pos<false>(il, t, nlines, ix.s0l, lo, probes);
                const uint32_t en = exact_pos<true>(ih, t, nlines, ix.s0l, hi, probes);
                const uint32_t m = en - st;
                if (m < best_m || (m == best_m && (uint32_t)k < best_k)) {
                    best_m = m; best_k = (uint32_t)k; best_st = st; best_en = en;
                }
            }
        }
    }
    const bool ring = valid && !full && !noprior && !by_bound && ix.K > 0 &&
                      (int64_t)best_m <= threshold;
    const bool dense = valid && !ring;
    if (ring) {                                  // for the ring scan
        w.rec[qq] = make_uint4(c, best_k, best_st, best_en);
        w.route[qq] = kRouteScan;
    }

    // ---- list appends: per-wave ballots, one atomic per list per block
    // (with fb.dense_masked the dense search reads the route codes instead
    // of a dense list; with KQ > 0 the ring queries stay in this block's
    // own list and no ring list is built)
    const unsigned long long rmask = __ballot(ring), dmask = __ballot(dense);
    if (lane == 0) {
        s_wcnt[wv][0] = (uint32_t)__popcll(rmask);
        s_wcnt[wv][1] = fb.dense_masked ? 0u : (uint32_t)__popcll(dmask);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t tot = 0;
        for (int i = 0; i < kWv; ++i) {
            const uint32_t c0 = s_wcnt[i][threadIdx.x];
            s_wcnt[i][threadIdx.x] = tot;
            tot += c0;
        }
        const bool global = threadIdx.x == 1 || KQ == 0;
        s_base[threadIdx.x] = global ? (tot ? atomicAdd(&w.counters[threadIdx.x], tot) : 0u) : tot;
    }
    __syncthreads();
    if (ring) {
        const uint32_t pos = s_wcnt[wv][0] + lane_prefix(rmask);
        if constexpr (KQ > 0) {
            s_rq[pos] = (uint32_t)qq;
            s_rr[pos] = make_uint4(c, best_k, best_st, best_en);
        } else {
            w.ring_list[s_base[0] + pos] = (uint32_t)qq;
        }
    }
    if (dense && !fb.dense_masked)
        w.dense_list[s_base[1] + s_wcnt[wv][1] + lane_prefix(dmask)] = (uint32_t)qq;

    // ---- statistics: wave sums, then one atomic per counter per block
    // full-search frames count as queries and dense queries only
    const unsigned long long v0 = wave_sum_u64(counted && !full && !by_bound ? best_m : 0);
    const unsigned long long v1 = wave_sum_u64(counted && !full && noprior ? 1 : 0);
    const unsigned long long bmask = __ballot(counted && by_bound);
    const unsigned long long v5 = wave_sum_u64(counted ? probes : 0u);
    const unsigned long long cdmask = __ballot(counted && dense);
    if (lane == 0) {
        s_st[wv][0] = v0;
        s_st[wv][1] = v1;
        s_st[wv][2] = (unsigned long long)__popcll(rmask);
        s_st[wv][3] = (unsigned long long)__popcll(cdmask);
        s_st[wv][4] = (unsigned long long)__popcll(bmask);
        s_st[wv][5] = v5;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned long long tot = 0;
        for (int i = 0; i < kWv; ++i) tot += s_st[i][threadIdx.x];
        const int slot[6] = {ST_MSTAR, ST_NOPRIOR, ST_RING, ST_DENSE, ST_BOUND, ST_PROBES};
        if (tot) stat_add(stats, slot[threadIdx.x], tot);
        if (threadIdx.x == 3 && !fb.dense_masked) {
            const int64_t nv = min<int64_t>(kBlk, Q - (int64_t)bx * kBlk);
            stat_add(stats, ST_QUERIES, (unsigned long long)nv);
        }
    }

    // ---- KQ > 0: this block's ring queries, one wavefront per query
    if constexpr (KQ > 0) {
        const uint32_t nring = s_base[0];
        unsigned long long surv = 0, mst = 0;
        for (uint32_t i = (uint32_t)wv; i < nring; i += kWv) {
            const uint4 rr = s_rr[i];
            const uint32_t t = scan_query<DP, KQ, 2>(ix, fb, w, s_rq[i], rr, lane);
            surv += t;
            mst += rr.w - rr.z;
        }
        if (nring) {
            if (lane == 0) { s_sc[wv][0] = surv; s_sc[wv][1] = mst; }
            __syncthreads();
            if (threadIdx.x < 2) {
                unsigned long long tot = 0;
                for (int i = 0; i < kWv; ++i) tot += s_sc[i][threadIdx.x];
                if (tot) stat_add(stats, threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING, tot);
            }
        }
    }
}

// ---------------------------------------------------------------- k_scan
// One wavefront per routed query; grid-strides over the ring list.  Every
// lane holds the query; lane k < K computes key k's ring bounds (lanes >= K
// hold [0, 2^32-1], which the zero padding of the pivot rows always meets);
// the filter reads them back with readlane at compile-time lane indices, so
// no LDS or barrier is used.  Each candidate's pivot row is read as Kp/4
// 16-byte loads issued together.
template <int DP>
__global__ __launch_bounds__(kBlock) void k_scan(DevIndex ix, FrameBatch fb, Work w,
                                                  unsigned long long *__restrict__ stats) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t count = w.counters[0];
    const uint32_t n = (uint32_t)ix.n;
    const int K = ix.K, kq = ix.Kp / 4;
    unsigned long long surv_tot = 0, mstar_tot = 0;
    for (uint32_t item = blockIdx.x * (kBlock / 64) + wv; item < count;
         item += gridDim.x * (kBlock / 64)) {
        const uint32_t qid = w.ring_list[item];
        const uint4 rec = w.rec[qid];
        const uint32_t c = rec.x, ks = rec.y, st = rec.z, en = rec.w;
        // lane i < DP/4 loads patch word i; readlane makes the words uniform
        const uint32_t mine = lane < DP / 4
            ? reinterpret_cast<const uint32_t *>(w.patches + (int64_t)qid * DP)[lane] : 0u;
        uint32_t a[DP / 4];
#pragma unroll
        for (int i = 0; i < DP / 4; ++i) a[i] = (uint32_t)__builtin_amdgcn_readlane((int)mine, i);
        const int Qc = w.qc[qid];
        uint32_t lo = 0, hi = 0xFFFFFFFFu;
        if (lane < K) {
            const int key = ix.keys[lane];
            int d = dot_row<DP>(a, ix.Rv + (int64_t)key * ix.Dp);
            uint32_t b = (uint32_t)(Qc + ix.Rc[key] + 2 * d);
            ring_bounds(b, c, lo, hi);
        }
        unsigned long long best = ~0ull;
        uint32_t cnt = 0;
        const int32_t *Pk = ix.P + (int64_t)ks * n;
        for (uint32_t j = st + lane; j < en; j += 64) {
            const int32_t r = Pk[j];
            const uint4 *row = reinterpret_cast<const uint4 *>(ix.Piv + (int64_t)r * ix.Kp);
            uint4 pv[kMaxKeys / 4];
#pragma unroll
            for (int q = 0; q < kMaxKeys / 4; ++q)
                if (q < kq) pv[q] = row[q];
            bool in = true;
#pragma unroll
            for (int q = 0; q < kMaxKeys / 4; ++q) {
                if (q < kq) {
                    const uint32_t x[4] = {pv[q].x, pv[q].y, pv[q].z, pv[q].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)lo, 4 * q + e);
                        const uint32_t hk = (uint32_t)__builtin_amdgcn_readlane((int)hi, 4 * q + e);
                        in = in && x[e] >= lk && x[e] <= hk;
                    }
                }
            }
            if (in) {
                ++cnt;
                int d = dot_row<DP>(a, ix.Rv + (int64_t)r * ix.Dp);
                const uint32_t s = (uint32_t)(Qc + ix.Rc[r] + 2 * d);
                const unsigned long long key = ((unsigned long long)s << 32) | (uint32_t)r;
                best = key < best ? key : best;
            }
        }
        best = wave_min_u64(best);
        const unsigned long long tot = wave_sum_u64(cnt);
        if (lane == 0) {
            const FrameDesc *fdp = &fb.f[w.fid[qid]];
            const int64_t ql = (int64_t)qid - fdp->qbase;
            fdp->out[ql] = (int32_t)(uint32_t)best;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(best >> 32);
            surv_tot += tot;
            mstar_tot += en - st;
        }
    }
    // one atomic per counter per block
    __shared__ unsigned long long s_acc[kBlock / 64][2];
    if (lane == 0) { s_acc[wv][0] = surv_tot; s_acc[wv][1] = mstar_tot; }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long tot = 0;
        for (int i = 0; i < kBlock / 64; ++i) tot += s_acc[i][threadIdx.x];
        if (tot) stat_add(stats, threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING, tot);
    }
}

// PivR[k][j] = Piv[P[k][j]], each row widened from Kp to KR words with zeros;
// entries j >= n (the list's padding to whole lines) are zero rows.
__global__ __launch_bounds__(256) void k_build_pivr(const uint32_t *__restrict__ Piv,
                                                     const int32_t *__restrict__ P, int64_t n,
                                                     int32_t n16, int32_t K, int32_t Kp,
                                                     int32_t KR, uint32_t *__restrict__ PivR) {
    const int64_t total = (int64_t)K * n16 * KR;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / KR;
        const int col = (int)(i - e * KR);
        const int k = (int)(e / n16);
        const int64_t j = e - (int64_t)k * n16;
        uint32_t v = 0;
        if (j < n && col < Kp) v = Piv[(int64_t)P[(int64_t)k * n + j] * Kp + col];
        PivR[i] = v;
    }
}

// ---------------------------------------------------------------- k_scan_knn
// k-NN variant of k_scan: each lane keeps the KN smallest (SSD, index) keys of
// its candidates in a sorted register list (KN = 2, 4 or 8 >= k); the
// wavefront then takes the global smallest by rounds of a wave minimum over
// the list heads (the keys are distinct: every candidate is scanned by one
// lane only) and writes the first k.
template <int DP, int KN>
__global__ __launch_bounds__(kBlock) void k_scan_knn(DevIndex ix, FrameBatch fb, Work w,
                                                      unsigned long long *__restrict__ stats) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t count = w.counters[0];
    const uint32_t n = (uint32_t)ix.n;
    const int K = ix.K, kq = ix.Kp / 4;
    unsigned long long surv_tot = 0, mstar_tot = 0;
    for (uint32_t item = blockIdx.x * (kBlock / 64) + wv; item < count;
         item += gridDim.x * (kBlock / 64)) {
        const uint32_t qid = w.ring_list[item];
        const uint4 rec = w.rec[qid];
        const uint32_t c = rec.x, ks = rec.y, st = rec.z, en = rec.w;
        const uint32_t mine = lane < DP / 4
            ? reinterpret_cast<const uint32_t *>(w.patches + (int64_t)qid * DP)[lane] : 0u;
        uint32_t a[DP / 4];
#pragma unroll
        for (int i = 0; i < DP / 4; ++i) a[i] = (uint32_t)__builtin_amdgcn_readlane((int)mine, i);
        const int Qc = w.qc[qid];
        uint32_t lo = 0, hi = 0xFFFFFFFFu;
        if (lane < K) {
            const int key = ix.keys[lane];
            int d = dot_row<DP>(a, ix.Rv + (int64_t)key * ix.Dp);
            uint32_t b = (uint32_t)(Qc + ix.Rc[key] + 2 * d);
            ring_bounds(b, c, lo, hi);
        }
        unsigned long long lst[KN];
#pragma unroll
        for (int j = 0; j < KN; ++j) lst[j] = ~0ull;
        uint32_t cnt = 0;
        const int32_t *Pk = ix.P + (int64_t)ks * n;
        for (uint32_t j = st + lane; j < en; j += 64) {
            const int32_t r = Pk[j];
            const uint4 *row = reinterpret_cast<const uint4 *>(ix.Piv + (int64_t)r * ix.Kp);
            uint4 pv[kMaxKeys / 4];
#pragma unroll
            for (int q = 0; q < kMaxKeys / 4; ++q)
                if (q < kq) pv[q] = row[q];
            bool in = true;
#pragma unroll
            for (int q = 0; q < kMaxKeys / 4; ++q) {
                if (q < kq) {
                    const uint32_t x[4] = {pv[q].x, pv[q].y, pv[q].z, pv[q].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)lo, 4 * q + e);
                        const uint32_t hk = (uint32_t)__builtin_amdgcn_readlane((int)hi, 4 * q + e);
                        in = in && x[e] >= lk && x[e] <= hk;
                    }
                }
            }
            if (in) {
                ++cnt;
                int d = dot_row<DP>(a, ix.Rv + (int64_t)r * ix.Dp);
                const uint32_t s = (uint32_t)(Qc + ix.Rc[r] + 2 * d);
                unsigned long long v = ((unsigned long long)s << 32) | (uint32_t)r;
#pragma unroll
                for (int q = 0; q < KN; ++q) {       // sorted insertion
                    const unsigned long long t = lst[q];
                    lst[q] = v < t ? v : t;
                    v = v < t ? t : v;
                }
            }
        }
        const FrameDesc *fdp = &fb.f[w.fid[qid]];
        const int64_t ql = (int64_t)qid - fdp->qbase;
#pragma unroll
        for (int r = 0; r < KN; ++r) {
            const unsigned long long m = wave_min_u64(lst[0]);
            if (lst[0] == m) {                       // the one lane holding it pops
#pragma unroll
                for (int q = 0; q + 1 < KN; ++q) lst[q] = lst[q + 1];
                lst[KN - 1] = ~0ull;
            }
            if (lane == 0 && r < fb.knn) {
                fdp->out[ql * fb.knn + r] = (int32_t)(uint32_t)m;
                if (fdp->ssd) fdp->ssd[ql * fb.knn + r] = (uint32_t)(m >> 32);
            }
        }
        const unsigned long long tot = wave_sum_u64(cnt);
        if (lane == 0) {
            surv_tot += tot;
            mstar_tot += en - st;
        }
    }
    __shared__ unsigned long long s_acc[kBlock / 64][2];
    if (lane == 0) { s_acc[wv][0] = surv_tot; s_acc[wv][1] = mstar_tot; }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long tot = 0;
        for (int i = 0; i < kBlock / 64; ++i) tot += s_acc[i][threadIdx.x];
        if (tot) stat_add(stats, threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING, tot);
    }
}

template <int DP, int KR, int KQ>
hipError_t launch_ring_kq(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          unsigned long long *stats, int64_t threshold, hipStream_t st) {
    const size_t lds = (size_t)ix.K * (ix.lbS + DP / 4 + 1) * 4;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ring<DP, KR, KQ>),
                       dim3((unsigned)((fb.Q + ring_block(KR) - 1) / ring_block(KR))),
                       dim3(ring_block(KR)), lds, st, ix, fb, w, stats, threshold);
    return hipGetLastError();
}

template <int DP, int KR>
hipError_t launch_ring_kr(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          unsigned long long *stats, int64_t threshold, hipStream_t st) {
    if (ring_scans_inline(ix, fb)) {
        switch (ix.KR) {
        case 8: return launch_ring_kq<DP, KR, 2>(ix, fb, w, stats, threshold, st);
        case 16: return launch_ring_kq<DP, KR, 4>(ix, fb, w, stats, threshold, st);
        }
        if constexpr (KR == 0) {
            switch (ix.KR) {
            case 32: return launch_ring_kq<DP, KR, 8>(ix, fb, w, stats, threshold, st);
            case 48: return launch_ring_kq<DP, KR, 12>(ix, fb, w, stats, threshold, st);
            case 64: return launch_ring_kq<DP, KR, 16>(ix, fb, w, stats, threshold, st);
            }
        }
        return hipErrorInvalidValue;
    }
    return launch_ring_kq<DP, KR, 0>(ix, fb, w, stats, threshold, st);
}

template <int DP>
hipError_t launch_ring_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                         unsigned long long *stats, int64_t threshold, hipStream_t st) {
    // the register-bound variant fits 80 VGPRs without spills up to Dp = 64
    if constexpr (DP <= 64) {
        if (ix.K <= 16) return launch_ring_kr<DP, 16>(ix, fb, w, stats, threshold, st);
    }
    return launch_ring_kr<DP, 0>(ix, fb, w, stats, threshold, st);
}

template <int DP>
hipError_t launch_scan_knn_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             unsigned long long *stats, hipStream_t st) {
    // lists of 2, 4 or 8 entries; the first fb.knn of them are written
    if (fb.knn < 2 || fb.knn > kMaxKnn) return hipErrorInvalidValue;
    if (fb.knn <= 2)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_knn<DP, 2>), dim3(1024), dim3(kBlock), 0, st,
                           ix, fb, w, stats);
    else if (fb.knn <= 4)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_knn<DP, 4>), dim3(1024), dim3(kBlock), 0, st,
                           ix, fb, w, stats);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_knn<DP, 8>), dim3(1024), dim3(kBlock), 0, st,
                           ix, fb, w, stats);
    return hipGetLastError();
}

template <int DP, int KQ>
hipError_t launch_scan_rows_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                              unsigned long long *stats, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_rows<DP, KQ>), dim3(1024), dim3(kBlock), 0, st, ix,
                       fb, w, stats);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_scan_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                         unsigned long long *stats, hipStream_t st) {
    if (ix.PivR) {
        switch (ix.KR) {
        case 8: return launch_scan_rows_t<DP, 2>(ix, fb, w, stats, st);
        case 16: return launch_scan_rows_t<DP, 4>(ix, fb, w, stats, st);
        case 32: return launch_scan_rows_t<DP, 8>(ix, fb, w, stats, st);
        case 48: return launch_scan_rows_t<DP, 12>(ix, fb, w, stats, st);
        case 64: return launch_scan_rows_t<DP, 16>(ix, fb, w, stats, st);
        default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<DP>), dim3(1024), dim3(kBlock), 0, st, ix, fb, w,
                       stats);
    return hipGetLastError();
}

}  // namespace

#define RIANN_DP_SWITCH(DPV, CALL)                 \
    switch (DPV) {                                 \
    case 32: return CALL(32);                      \
    case 64: return CALL(64);                      \
    case 96: return CALL(96);                      \
    case 128: return CALL(128);                    \
    case 160: return CALL(160);                    \
    case 192: return CALL(192);                    \
    case 224: return CALL(224);                    \
    case 256: return CALL(256);                    \
    default: return hipErrorInvalidValue;          \
    }

hipError_t launch_ring(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                       unsigned long long *stats, int64_t threshold, hipStream_t st) {
#define CALL_RING(D) launch_ring_t<D>(ix, fb, w, stats, threshold, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_RING)
#undef CALL_RING
}

hipError_t launch_scan(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                       unsigned long long *stats, hipStream_t st) {
#define CALL_SCAN(D) launch_scan_t<D>(ix, fb, w, stats, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_SCAN)
#undef CALL_SCAN
}

int pivr_words(int K) { return K <= 8 ? 8 : (K + 15) / 16 * 16; }

bool ring_scans_inline(const DevIndex &ix, const FrameBatch &fb) {
    return fb.dense_masked && fb.knn == 1 && ix.PivR != nullptr && ix.K > 0;
}

hipError_t launch_build_pivr(const DevIndex &ix, uint32_t *PivR, hipStream_t st) {
    const int64_t total = (int64_t)ix.K * ix.n16 * pivr_words(ix.K);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_build_pivr, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                       ix.Piv, ix.P, ix.n, ix.n16, ix.K, ix.Kp, pivr_words(ix.K), PivR);
    return hipGetLastError();
}

hipError_t launch_scan_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                           unsigned long long *stats, hipStream_t st) {
#define CALL_SCAN_KNN(D) launch_scan_knn_t<D>(ix, fb, w, stats, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_SCAN_KNN)
#undef CALL_SCAN_KNN
}

}  // namespace riann
