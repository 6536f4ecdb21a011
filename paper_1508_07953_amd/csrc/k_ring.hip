// k_ring.hip -- ring phase and ring scan of the exact-mode RIANN search.
//
// k_ring (one lane per query) follows the per-query steps of Algorithm 1:
//   extract q; c = SSD(q, R[prev]) (radius^2 from the previous match);
//   b_k = SSD(q, key_k); ring k = [lo_k, hi_k] in key-distance space with
//   integer bounds (no rounding slack); two binary searches in key k's
//   sorted list give [st_k, en_k) (Sec. 3.3: "two binary searches"); the
//   smallest ring k* is kept; the query is routed to the ring scan when
//   m* = en - st is small and to the dense search otherwise.
// k_scan (one wavefront per routed query) scans key k*'s ring, keeps the
//   references inside all K rings (the intersection S) and takes the argmin
//   of the exact SSD over S with a wavefront reduction (lowest index on ties).
#include "riann_internal.h"

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

// <a, v> over DP bytes: a in registers, v a 16-byte aligned reference row.
template <int DP>
__device__ __forceinline__ int dot_row(const uint32_t (&a)[DP / 4], const int8_t *__restrict__ v) {
    const uint4 *v4 = reinterpret_cast<const uint4 *>(v);
    int acc = 0;
#pragma unroll
    for (int i = 0; i < DP / 16; ++i) {
        uint4 r = v4[i];
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 0], (int)r.x, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 1], (int)r.y, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 2], (int)r.z, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 3], (int)r.w, acc, false);
    }
    return acc;
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
// sample_count searches the list's samples in LDS (S[i] = T[16 s0l i], ns of
// them) and returns how many satisfy the predicate; that brackets the
// position (pos_bracket).  exact_pos finishes the search in global memory:
// a binary search over the first entries of 16-entry lines, then one
// aligned 64-byte line is read and counted.
template <bool LE>
__device__ __forceinline__ bool pred(uint32_t x, uint32_t v) { return LE ? x <= v : x < v; }

template <bool LE>
__device__ __forceinline__ int sample_count(const uint32_t *S, int ns, uint32_t v) {
    int lo = 0, len = ns;
    while (len > 0) {
        const int half = len >> 1;
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
                                              int s0l, uint32_t v) {
    if (i == 0) return 0;
    int L = (i - 1) * s0l, H = min(i * s0l, nlines);
    while (H - L > 1) {
        const int mid = (L + H) >> 1;
        if (pred<LE>(T[16 * mid], v)) L = mid;
        else H = mid;
    }
    const uint4 *line = reinterpret_cast<const uint4 *>(T + 16 * L);
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 x = line[q];
        cnt += pred<LE>(x.x, v) + pred<LE>(x.y, v) + pred<LE>(x.z, v) + pred<LE>(x.w, v);
    }
    return 16u * (uint32_t)L + cnt;
}

__device__ __forceinline__ uint32_t lane_prefix(unsigned long long mask) {
    unsigned m = __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u);
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), m);
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- k_ring
// One lane per query, 1024 queries per block.  Each block first copies the
// binary-search samples of all K lists (at most 64 KB) into LDS.  For every
// key the LDS samples bracket the ring size m_k to an interval [ml, mh]; the
// exact size (two line reads in global memory) is computed only for keys
// that can still be the smallest ring: key k is skipped when ml > min over
// earlier keys of mh (some earlier ring is strictly smaller) or ml >= the
// smallest exact size so far (an earlier key wins the tie).  The result --
// the exact smallest ring m*, its key k* (lowest on ties) and its range --
// is the same as evaluating every key exactly.
// List appends and statistics are aggregated per block: one atomic per list
// and per counter per block.
constexpr int kRingBlock = 1024;
constexpr int kRingWaves = kRingBlock / 64;

template <int DP>
__global__ __launch_bounds__(kRingBlock) void k_ring(DevIndex ix, FrameBatch fb, Work w,
                                                      unsigned long long *__restrict__ stats,
                                                      int64_t threshold) {
    extern __shared__ __attribute__((aligned(16))) uint32_t s_samp[];
    __shared__ uint32_t s_wcnt[kRingWaves][2];
    __shared__ uint32_t s_base[2];
    __shared__ unsigned long long s_st[kRingWaves][4];
    const int nsamp = ix.K * ix.ns;
    // 16-byte copies (the table is 256-byte aligned): four rounds for 64 KB
    for (int i = threadIdx.x; i < nsamp / 4; i += kRingBlock)
        reinterpret_cast<uint4 *>(s_samp)[i] = reinterpret_cast<const uint4 *>(ix.Ts)[i];
    for (int i = (nsamp & ~3) + threadIdx.x; i < nsamp; i += kRingBlock) s_samp[i] = ix.Ts[i];
    __syncthreads();

    const int64_t Q = fb.Q;
    const uint32_t n = (uint32_t)ix.n;
    const int nlines = ix.n16 / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t qid = (int64_t)blockIdx.x * kRingBlock + threadIdx.x;
    const bool valid = qid < Q;
    const int64_t qq = valid ? qid : Q - 1;
    const FrameDesc *fdp = &fb.f[w.fid[qq]];
    const bool full = fdp->mode == kModeFull;
    const int32_t *prev = full ? nullptr : fdp->prev;
    const int64_t ql = qq - fdp->qbase;
    uint32_t a[DP / 4];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(w.patches + qq * DP);
#pragma unroll
        for (int i = 0; i < DP / 16; ++i) {
            const uint4 v = src[i];
            a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
        }
    }
    const int Qc = w.qc[qq];
    // radius: the SSD to the previous match; for k-NN fields the largest SSD
    // to the k previous matches, which must be k distinct references (then
    // the k nearest lie within it); anything else means no prior
    bool noprior = prev == nullptr;
    uint32_t c = 0xFFFFFFFFu;
    if (!noprior) {
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
    if (!full && !noprior && ix.K > 0) {
        uint32_t up = 0xFFFFFFFFu;        // min over evaluated keys of mh
        bool have = false;                // best_m holds an exact size
        for (int k = 0; k < ix.K; ++k) {
            const int key = ix.keys[k];
            int d = dot_row<DP>(a, ix.Rv + (int64_t)key * ix.Dp);
            uint32_t b = (uint32_t)(Qc + ix.Rc[key] + 2 * d);
            uint32_t lo, hi;
            ring_bounds(b, c, lo, hi);
            const uint32_t *S = s_samp + k * ix.ns;
            const int il = sample_count<false>(S, ix.ns, lo);
            const int ih = sample_count<true>(S, ix.ns, hi);
            uint32_t sl, sh, el, eh;
            pos_bracket(il, ix.ns, ix.s0l, n, sl, sh);
            pos_bracket(ih, ix.ns, ix.s0l, n, el, eh);
            const uint32_t ml = el > sh ? el - sh : 0u, mh = eh - sl;
            if (ml > up || (have && ml >= best_m)) continue;
            up = min(up, mh);
            const uint32_t *t = ix.T + (int64_t)k * ix.n16;
            const uint32_t st = exact_pos<false>(il, t, nlines, ix.s0l, lo);
            const uint32_t en = exact_pos<true>(ih, t, nlines, ix.s0l, hi);
            const uint32_t m = en - st;
            if (!have || m < best_m) { best_m = m; best_k = k; best_st = st; best_en = en; have = true; }
        }
    }
    const bool ring = valid && !full && !noprior && ix.K > 0 && (int64_t)best_m <= threshold;
    const bool dense = valid && !ring;
    if (valid) w.rec[qq] = make_uint4(c, best_k, best_st, best_en);

    // ---- list appends: per-wave ballots, one atomic per list per block
    const unsigned long long rmask = __ballot(ring), dmask = __ballot(dense);
    if (lane == 0) {
        s_wcnt[wv][0] = (uint32_t)__popcll(rmask);
        s_wcnt[wv][1] = (uint32_t)__popcll(dmask);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t tot = 0;
        for (int i = 0; i < kRingWaves; ++i) {
            const uint32_t c0 = s_wcnt[i][threadIdx.x];
            s_wcnt[i][threadIdx.x] = tot;
            tot += c0;
        }
        s_base[threadIdx.x] = tot ? atomicAdd(&w.counters[threadIdx.x], tot) : 0u;
    }
    __syncthreads();
    if (ring) w.ring_list[s_base[0] + s_wcnt[wv][0] + lane_prefix(rmask)] = (uint32_t)qq;
    if (dense) w.dense_list[s_base[1] + s_wcnt[wv][1] + lane_prefix(dmask)] = (uint32_t)qq;

    // ---- statistics: wave sums, then one atomic per counter per block
    // full-search frames count as queries and dense queries only
    const unsigned long long v0 = wave_sum_u64(valid && !full ? best_m : 0);
    const unsigned long long v1 = wave_sum_u64(valid && !full && noprior ? 1 : 0);
    if (lane == 0) {
        s_st[wv][0] = v0;
        s_st[wv][1] = v1;
        s_st[wv][2] = (unsigned long long)__popcll(rmask);
        s_st[wv][3] = (unsigned long long)__popcll(dmask);
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long tot = 0;
        for (int i = 0; i < kRingWaves; ++i) tot += s_st[i][threadIdx.x];
        const int slot[4] = {ST_MSTAR, ST_NOPRIOR, ST_RING, ST_DENSE};
        if (tot) atomicAdd(&stats[slot[threadIdx.x]], tot);
        if (threadIdx.x == 3) {
            const int64_t nv = min<int64_t>(kRingBlock, Q - (int64_t)blockIdx.x * kRingBlock);
            atomicAdd(&stats[ST_QUERIES], (unsigned long long)nv);
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
        if (tot) atomicAdd(&stats[threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING], tot);
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
        if (tot) atomicAdd(&stats[threadIdx.x == 0 ? ST_SURV : ST_MSTAR_RING], tot);
    }
}

template <int DP>
hipError_t launch_ring_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                         unsigned long long *stats, int64_t threshold, hipStream_t st) {
    const int64_t blocks = (fb.Q + kRingBlock - 1) / kRingBlock;
    const size_t lds = (size_t)ix.K * ix.ns * 4;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ring<DP>), dim3((unsigned)blocks), dim3(kRingBlock),
                       lds, st, ix, fb, w, stats, threshold);
    return hipGetLastError();
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

template <int DP>
hipError_t launch_scan_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                         unsigned long long *stats, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<DP>), dim3(1024), dim3(kBlock), 0, st, ix, fb, w,
                       stats);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

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

hipError_t launch_scan_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                           unsigned long long *stats, hipStream_t st) {
#define CALL_SCAN_KNN(D) launch_scan_knn_t<D>(ix, fb, w, stats, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_SCAN_KNN)
#undef CALL_SCAN_KNN
}

}  // namespace riann
