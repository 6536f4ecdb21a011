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

// Loads the D patch bytes of the window with top-left pixel (x, y) into
// packed words, each byte XOR-ed with `xorv`; bytes k >= D are 0.
template <int DP>
__device__ __forceinline__ void load_patch(const uint8_t *__restrict__ frame, int64_t pitch,
                                           int x, int y, int C, int rowlen, int D,
                                           uint32_t xorv, uint32_t (&w)[DP / 4]) {
    const uint8_t *row = frame + (int64_t)y * pitch + (int64_t)x * C;
    int rem = 0;
#pragma unroll
    for (int i = 0; i < DP / 4; ++i) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 4 * i + b;
            if (k < D) word |= ((uint32_t)row[rem] ^ xorv) << (8 * b);
            if (++rem == rowlen) { rem = 0; row += pitch; }
        }
        w[i] = word;
    }
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

// first j in [0, n) with t[j] >= v
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *__restrict__ t, uint32_t n,
                                                    uint32_t v) {
    uint32_t lo = 0, len = n;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (t[lo + half] < v) { lo += half + 1; len -= half + 1; }
        else len = half;
    }
    return lo;
}

// first j in [0, n) with t[j] > v
__device__ __forceinline__ uint32_t upper_bound_u32(const uint32_t *__restrict__ t, uint32_t n,
                                                    uint32_t v) {
    uint32_t lo = 0, len = n;
    while (len > 0) {
        uint32_t half = len >> 1;
        if (t[lo + half] <= v) { lo += half + 1; len -= half + 1; }
        else len = half;
    }
    return lo;
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
template <int DP>
__global__ __launch_bounds__(kBlock) void k_ring(DevIndex ix, FrameArgs fa,
                                                  const int32_t *__restrict__ prev, Work w,
                                                  unsigned long long *__restrict__ stats,
                                                  int64_t threshold) {
    const int64_t Q = (int64_t)fa.Hq * fa.Wq;
    const int64_t qid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = qid < Q;
    const int64_t qq = valid ? qid : Q - 1;
    const int qi = (int)(qq / fa.Wq), qj = (int)(qq % fa.Wq);
    uint32_t a[DP / 4];
    load_patch<DP>(fa.frame, fa.pitch, qj * ix.s, qi * ix.s, ix.C, ix.p * ix.C, ix.D, 0x7Fu, a);
    // Qc = sum (a+1)^2 = sum a^2 + 2 sum a + D
    int sa2 = 0, sa = 0;
#pragma unroll
    for (int i = 0; i < DP / 4; ++i) {
        sa2 = __builtin_amdgcn_sdot4((int)a[i], (int)a[i], sa2, false);
        sa = __builtin_amdgcn_sdot4((int)a[i], 0x01010101, sa, false);
    }
    const int Qc = sa2 + 2 * sa + ix.D;

    const int32_t pv = prev ? prev[qq] : -1;
    const bool noprior = pv < 0 || (int64_t)pv >= ix.n;
    uint32_t c = 0xFFFFFFFFu;
    if (!noprior) {
        int d = dot_row<DP>(a, ix.Rv + (int64_t)pv * ix.Dp);
        c = (uint32_t)(Qc + ix.Rc[pv] + 2 * d);
    }
    const uint32_t n = (uint32_t)ix.n;
    uint32_t best_m = n, best_k = 0, best_st = 0, best_en = n;
    if (!noprior) {
        for (int k = 0; k < ix.K; ++k) {
            const int key = ix.keys[k];
            int d = dot_row<DP>(a, ix.Rv + (int64_t)key * ix.Dp);
            uint32_t b = (uint32_t)(Qc + ix.Rc[key] + 2 * d);
            uint32_t lo, hi;
            ring_bounds(b, c, lo, hi);
            const uint32_t *t = ix.T + (int64_t)k * n;
            uint32_t st = lower_bound_u32(t, n, lo);
            uint32_t en = upper_bound_u32(t, n, hi);
            uint32_t m = en - st;
            if (m < best_m) { best_m = m; best_k = k; best_st = st; best_en = en; }
        }
    }
    const bool ring = valid && !noprior && ix.K > 0 && (int64_t)best_m <= threshold;
    const bool dense = valid && !ring;
    if (valid) w.rec[qq] = make_uint4(c, best_k, best_st, best_en);

    // append to the ring / dense lists, one atomic per wavefront and list
    const unsigned long long rmask = __ballot(ring), dmask = __ballot(dense);
    const int lane = threadIdx.x & 63;
    uint32_t rbase = 0, dbase = 0;
    if (lane == 0) {
        if (rmask) rbase = atomicAdd(&w.counters[0], (uint32_t)__popcll(rmask));
        if (dmask) dbase = atomicAdd(&w.counters[1], (uint32_t)__popcll(dmask));
    }
    rbase = __shfl(rbase, 0, 64);
    dbase = __shfl(dbase, 0, 64);
    if (ring) w.ring_list[rbase + lane_prefix(rmask)] = (uint32_t)qq;
    if (dense) w.dense_list[dbase + lane_prefix(dmask)] = (uint32_t)qq;

    unsigned long long ms = valid ? best_m : 0, np = (valid && noprior) ? 1 : 0;
    ms = wave_sum_u64(ms);
    np = wave_sum_u64(np);
    const unsigned long long nv = __popcll(__ballot(valid));
    if (lane == 0) {
        atomicAdd(&stats[ST_QUERIES], nv);
        atomicAdd(&stats[ST_RING], (unsigned long long)__popcll(rmask));
        atomicAdd(&stats[ST_DENSE], (unsigned long long)__popcll(dmask));
        atomicAdd(&stats[ST_NOPRIOR], np);
        atomicAdd(&stats[ST_MSTAR], ms);
    }
}

// ---------------------------------------------------------------- k_scan
// One wavefront per routed query; grid-strides over the ring list.  Every
// lane holds the query; lane k < K computes key k's ring bounds, which the
// filter reads back with readlane (uniform k), so no LDS or barrier is used.
template <int DP>
__global__ __launch_bounds__(kBlock) void k_scan(DevIndex ix, FrameArgs fa, Work w,
                                                  int32_t *__restrict__ out,
                                                  uint32_t *__restrict__ ssd,
                                                  unsigned long long *__restrict__ stats) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t count = w.counters[0];
    const uint32_t n = (uint32_t)ix.n;
    const int K = ix.K;
    unsigned long long surv_tot = 0, mstar_tot = 0;
    for (uint32_t item = blockIdx.x * (kBlock / 64) + wv; item < count;
         item += gridDim.x * (kBlock / 64)) {
        const uint32_t qid = w.ring_list[item];
        const uint4 rec = w.rec[qid];
        const uint32_t c = rec.x, ks = rec.y, st = rec.z, en = rec.w;
        const int qi = (int)(qid / (uint32_t)fa.Wq), qj = (int)(qid % (uint32_t)fa.Wq);
        uint32_t a[DP / 4];
        load_patch<DP>(fa.frame, fa.pitch, qj * ix.s, qi * ix.s, ix.C, ix.p * ix.C, ix.D,
                       0x7Fu, a);
        int sa2 = 0, sa = 0;
#pragma unroll
        for (int i = 0; i < DP / 4; ++i) {
            sa2 = __builtin_amdgcn_sdot4((int)a[i], (int)a[i], sa2, false);
            sa = __builtin_amdgcn_sdot4((int)a[i], 0x01010101, sa, false);
        }
        const int Qc = sa2 + 2 * sa + ix.D;
        uint32_t lo = 0, hi = 0;
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
            const uint32_t *row = ix.Piv + (int64_t)r * K;
            bool in = true;
            for (int k = 0; k < K; ++k) {
                const uint32_t v = row[k];
                const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)lo, k);
                const uint32_t hk = (uint32_t)__builtin_amdgcn_readlane((int)hi, k);
                in = in && v >= lk && v <= hk;
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
            out[qid] = (int32_t)(uint32_t)best;
            if (ssd) ssd[qid] = (uint32_t)(best >> 32);
            surv_tot += tot;
            mstar_tot += en - st;
        }
    }
    if (lane == 0 && (surv_tot | mstar_tot)) {
        atomicAdd(&stats[ST_SURV], surv_tot);
        atomicAdd(&stats[ST_MSTAR_RING], mstar_tot);
    }
}

template <int DP>
hipError_t launch_ring_t(const DevIndex &ix, const FrameArgs &fa, const int32_t *prev,
                         const Work &w, unsigned long long *stats, int64_t threshold,
                         hipStream_t st) {
    const int64_t Q = (int64_t)fa.Hq * fa.Wq;
    const int blocks = (int)((Q + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ring<DP>), dim3(blocks), dim3(kBlock), 0, st, ix, fa,
                       prev, w, stats, threshold);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_scan_t(const DevIndex &ix, const FrameArgs &fa, const Work &w, int32_t *out,
                         uint32_t *ssd, unsigned long long *stats, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<DP>), dim3(1024), dim3(kBlock), 0, st, ix, fa, w,
                       out, ssd, stats);
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

hipError_t launch_ring(const DevIndex &ix, const FrameArgs &fa, const int32_t *prev,
                       const Work &w, unsigned long long *stats, int64_t threshold,
                       hipStream_t st) {
#define CALL_RING(D) launch_ring_t<D>(ix, fa, prev, w, stats, threshold, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_RING)
#undef CALL_RING
}

hipError_t launch_scan(const DevIndex &ix, const FrameArgs &fa, const Work &w, int32_t *out,
                       uint32_t *ssd, unsigned long long *stats, hipStream_t st) {
#define CALL_SCAN(D) launch_scan_t<D>(ix, fa, w, out, ssd, stats, st)
    RIANN_DP_SWITCH(ix.Dp, CALL_SCAN)
#undef CALL_SCAN
}

}  // namespace riann
