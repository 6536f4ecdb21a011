// k_paper.hip -- the paper's own approximate search (Algorithm 1): fat rings
// d -/+ alpha*d (alpha = 1/4) around the previous match, then around random
// anchors drawn from the candidate set until fewer than L candidates remain.
//
// One wavefront per query.  The first ring is a contiguous range of the
// previous match's sorted distance row (two 64-ary searches), so the
// candidate set S is a bit mask over that range's positions, plus a flag for
// the previous match itself, kept in LDS; "already an anchor" is a second
// mask.  Each anchor's ring filters the set 64 positions at a time: lane l
// tests position b + l (candidate index from the sorted row, its distance to
// the anchor from the n x n matrix) and a ballot gives the new 64 bits.
// Anchors are drawn with the counter-based SplitMix64 chain of
// (seed, frame, query, iteration), as the u-th member not yet drawn, in the
// set's order (previous match first, then row order).  In squared integer
// distances the ring test is 9c <= 16a <= 25c.
#include "riann_internal.h"

namespace riann {

namespace {

constexpr int kPWaves = 4;

__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t t, uint64_t q, uint64_t it) {
    return splitmix(splitmix(splitmix(splitmix(seed) ^ t) ^ q) ^ it);
}

__device__ __forceinline__ bool in_ring(uint32_t a, uint64_t c) {
    const uint64_t a16 = 16ull * a;
    return 9ull * c <= a16 && a16 <= 25ull * c;
}

template <int DP>
__device__ __forceinline__ int dot_q(const uint32_t (&a)[DP / 4], const int8_t *__restrict__ v) {
    const uint4 *p = reinterpret_cast<const uint4 *>(v);
    int d = 0;
#pragma unroll
    for (int i = 0; i < DP / 16; ++i) {
        const uint4 x = p[i];
        d = __builtin_amdgcn_sdot4((int)a[4 * i], (int)x.x, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 1], (int)x.y, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 2], (int)x.z, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 3], (int)x.w, d, false);
    }
    return d;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)v, m, 64);
        const unsigned hi = __shfl_xor((unsigned)(v >> 32), m, 64);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

// First position p in [lo, hi) of a monotone (false...true) predicate over a
// sorted row, hi when none: 64-ary narrowing, one probe per lane per step.
template <class Pred>
__device__ __forceinline__ int64_t first_true(int64_t lo, int64_t hi, int lane, Pred pred) {
    while (hi - lo > 64) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t pos = lo + (int64_t)lane * step;
        const bool t = pos < hi ? pred(pos) : true;
        const unsigned long long mask = __ballot(t);
        const int f = mask ? __builtin_ctzll(mask) : 64;
        if (f == 0) return lo;                      // pred(lo) holds
        const int64_t left = lo + (int64_t)(f - 1) * step;   // pred false here
        const int64_t right = f < 64 ? min(hi, lo + (int64_t)f * step) : hi;
        lo = left + 1;
        hi = right;
    }
    const int64_t pos = lo + lane;
    const bool t = pos < hi ? pred(pos) : false;
    const unsigned long long mask = __ballot(t);
    return mask ? lo + __builtin_ctzll(mask) : hi;
}

template <int DP>
__global__ __launch_bounds__(64 * kPWaves) void k_paper(DevIndex ix, FrameBatch fb, Work w,
                                                        PaperArgs pa) {
    extern __shared__ uint32_t s_masks[];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n = ix.n;
    const int nw = (int)((n + 31) / 32) + 2;
    uint32_t *Sm = s_masks + (int64_t)wv * 3 * nw, *Um = Sm + nw, *Nm = Um + nw;
    const int64_t Q = fb.Q;
    for (int64_t qid = (int64_t)blockIdx.x * kPWaves + wv; qid < Q;
         qid += (int64_t)gridDim.x * kPWaves) {
        const FrameDesc *fdp = &fb.f[w.fid[qid]];
        const int64_t ql = qid - fdp->qbase;
        const uint32_t mine = lane < DP / 4
            ? reinterpret_cast<const uint32_t *>(w.patches + qid * DP)[lane] : 0u;
        uint32_t a[DP / 4];
#pragma unroll
        for (int i = 0; i < DP / 4; ++i) a[i] = (uint32_t)__builtin_amdgcn_readlane((int)mine, i);
        const int Qc = w.qc[qid];
        // previous match; an entry outside [0, n) draws a random one
        int64_t ri = fdp->prev ? fdp->prev[ql] : -1;
        if (ri < 0 || ri >= n) ri = (int64_t)(draw(pa.seed, pa.t, (uint64_t)ql, 0xFFFFFFFFull) %
                                              (uint64_t)n);
        const uint64_t c = (uint32_t)(Qc + ix.Rc[ri] + 2 * dot_q<DP>(a, ix.Rv + ri * ix.Dp));
        // the fat ring of r_i: positions [st, en) of its sorted row
        const uint32_t *row = pa.T + ri * n;
        const int64_t st = first_true(0, n, lane, [&](int64_t p) { return 16ull * row[p] >= 9ull * c; });
        const int64_t en = first_true(st, n, lane, [&](int64_t p) { return 16ull * row[p] > 25ull * c; });
        const int64_t m0 = en - st;
        const int mw = (int)((m0 + 31) / 32);
        for (int k = lane; k < mw + 2; k += 64) {
            uint32_t v = 0;
            if (k < mw) v = (k < mw - 1 || (m0 & 31) == 0) ? ~0u : ((1u << (m0 & 31)) - 1u);
            Sm[k] = v;
            Um[k] = 0u;
        }
        bool fS = c > 0, fU = false;                  // r_i as a member, and drawn
        int64_t size = m0 + (fS ? 1 : 0);
        const int32_t *prow = pa.P + ri * n + st;
        int32_t it = 0;
        for (;;) {
            if (size < pa.L) break;
            // members not yet drawn
            uint32_t fc = 0;
            for (int k = lane; k < mw; k += 64) fc += (uint32_t)__popc(Sm[k] & ~Um[k]);
            const uint64_t nfree = (uint64_t)wave_sum(fc) + ((fS && !fU) ? 1u : 0u);
            if (nfree == 0) break;
            uint64_t u = draw(pa.seed, pa.t, (uint64_t)ql, (uint64_t)it) % nfree;
            int64_t rk;
            if (fS && !fU && u == 0) {
                rk = ri;
                fU = true;
            } else {
                if (fS && !fU) u -= 1;
                // u-th free position: per-lane chunks of words, wave prefix sums
                const int chunk = (mw + 63) / 64;
                const int w0 = lane * chunk, w1 = min(mw, w0 + chunk);
                uint32_t cnt = 0;
                for (int k = w0; k < w1; ++k) cnt += (uint32_t)__popc(Sm[k] & ~Um[k]);
                uint32_t incl = cnt;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
                    if (lane >= o) incl += y;
                }
                const unsigned long long owner = __ballot((uint64_t)incl > u);
                const int L0 = __builtin_ctzll(owner);
                int64_t pos = 0;
                if (lane == L0) {
                    uint64_t rem = u - (uint64_t)(incl - cnt);
                    for (int k = w0; k < w1; ++k) {
                        uint32_t f = Sm[k] & ~Um[k];
                        const uint32_t pc = (uint32_t)__popc(f);
                        if (rem < pc) {
                            for (uint64_t r = 0; r < rem; ++r) f &= f - 1;   // drop lower bits
                            pos = (int64_t)k * 32 + __builtin_ctz(f);
                            break;
                        }
                        rem -= pc;
                    }
                    Um[pos >> 5] |= 1u << (pos & 31);
                }
                pos = ((int64_t)__shfl((int)(pos >> 32), L0, 64) << 32) |
                      (uint32_t)__shfl((int)pos, L0, 64);
                rk = prow[pos];
            }
            ++it;
            const uint64_t ck =
                (uint32_t)(Qc + ix.Rc[rk] + 2 * dot_q<DP>(a, ix.Rv + rk * ix.Dp));
            const uint32_t *drow = pa.Dm + rk * n;
            // filter S by the anchor's ring into Nm; keep S when nothing survives
            uint32_t kept = 0;
            for (int64_t b = 0; b < m0; b += 64) {
                const int k = (int)(b >> 5);
                const uint32_t s0 = Sm[k], s1 = Sm[k + 1];
                if ((s0 | s1) == 0) {
                    if (lane == 0) { Nm[k] = 0u; Nm[k + 1] = 0u; }
                    continue;
                }
                const int64_t pos = b + lane;
                const bool in = ((lane < 32 ? s0 >> lane : s1 >> (lane - 32)) & 1u) != 0;
                const bool keep = in && in_ring(drow[prow[pos]], ck);
                const unsigned long long nm = __ballot(keep);
                if (lane == 0) {
                    Nm[k] = (uint32_t)nm;
                    Nm[k + 1] = (uint32_t)(nm >> 32);
                }
                kept += (uint32_t)__popcll(nm);
            }
            const bool keepF = fS && in_ring(drow[ri], ck);
            const int64_t total = (int64_t)kept + (keepF ? 1 : 0);
            if (total == 0) break;                     // the ring would empty S
            for (int k = lane; k < mw; k += 64) Sm[k] = Nm[k];
            fS = keepF;
            size = total;
        }
        // (SSD, index) minimum over S
        unsigned long long best = fS ? ((c << 32) | (uint64_t)ri) : ~0ull;
        for (int64_t b = 0; b < m0; b += 64) {
            const int k = (int)(b >> 5);
            const uint32_t s0 = Sm[k], s1 = Sm[k + 1];
            if ((s0 | s1) == 0) continue;
            const bool in = ((lane < 32 ? s0 >> lane : s1 >> (lane - 32)) & 1u) != 0;
            if (in) {
                const int64_t j = prow[b + lane];
                const uint32_t s = (uint32_t)(Qc + ix.Rc[j] + 2 * dot_q<DP>(a, ix.Rv + j * ix.Dp));
                const unsigned long long key = ((unsigned long long)s << 32) | (uint64_t)j;
                best = key < best ? key : best;
            }
        }
        best = wave_min64(best);
        if (lane == 0) {
            fdp->out[ql] = (int32_t)(uint32_t)best;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(best >> 32);
            if (pa.iters) pa.iters[ql] = it;
        }
    }
}

}  // namespace

size_t paper_lds_bytes(int64_t n) {
    return (size_t)kPWaves * 3 * (size_t)((n + 31) / 32 + 2) * 4;
}

hipError_t launch_paper(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                        const PaperArgs &pa, hipStream_t st) {
    const int64_t want = (fb.Q + kPWaves - 1) / kPWaves;
    const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 65536 ? 65536 : want));
    const size_t lds = paper_lds_bytes(ix.n);
#define RIANN_PAPER(D)                                                                        \
    case D:                                                                                   \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_paper<D>), dim3(blocks), dim3(64 * kPWaves), lds, \
                           st, ix, fb, w, pa);                                                \
        break;
    switch (ix.Dp) {
        RIANN_PAPER(32) RIANN_PAPER(64) RIANN_PAPER(96) RIANN_PAPER(128)
        RIANN_PAPER(160) RIANN_PAPER(192) RIANN_PAPER(224) RIANN_PAPER(256)
    default: return hipErrorInvalidValue;
    }
#undef RIANN_PAPER
    return hipGetLastError();
}

}  // namespace riann
