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
// it.  A resolve kernel then recomputes that one tile's 32 exact SSDs and
// takes their (SSD, index) minimum -- the global one, because every row
// outside the tile has a larger Y, hence a larger SSD (2Y + p grows with Y).
// When the smallest Y occurs in two different tiles the parities of those
// tiles could decide differently, so such a query is handed to the
// column-layout kernel (its index is appended to the fallback list).
#include "riann_internal.h"

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

constexpr int kWaves = 8;
constexpr int kBlock = 64 * kWaves;
constexpr int kQB = 2;                 // 32-query column blocks per wavefront
constexpr int kWaveQ = 32 * kQB;
constexpr int kBlockQ = kWaveQ * kWaves;
constexpr int kTPS = 2;                // tiles per step

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
    uint32_t tie[kQB];      // another tile reached the same Y

    __device__ __forceinline__ void load_step(const int8_t *lf, const int32_t *lh, int u,
                                              int lane, int grp, v4i (&Af)[kTPS][KB],
                                              v16i (&H)[kTPS]) {
#pragma unroll
        for (int v = 0; v < kTPS; ++v) {
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                Af[v][kb] = *reinterpret_cast<const v4i *>(lf + ((u * kTPS + v) * KB + kb) * 1024 +
                                                           lane * 16);
            const v4i *hp = reinterpret_cast<const v4i *>(lh + (u * kTPS + v) * kTile + grp * 16);
            const v4i h0 = hp[0], h1 = hp[1], h2 = hp[2], h3 = hp[3];
            H[v] = v16i{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3],
                        h2[0], h2[1], h2[2], h2[3], h3[0], h3[1], h3[2], h3[3]};
        }
    }

    __device__ __forceinline__ void mma(int qb, const v4i (&Af)[kTPS][KB], const v16i (&H)[kTPS],
                                        v16i (&acc)[kTPS]) {
#pragma unroll
        for (int v = 0; v < kTPS; ++v) {
            acc[v] = H[v];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                acc[v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[v][kb], Bq[qb][kb], acc[v], 0, 0,
                                                               0);
        }
    }

    __device__ __forceinline__ void track(int qb, const v16i (&acc)[kTPS], uint32_t t0) {
#pragma unroll
        for (int v = 0; v < kTPS; ++v) {
            const uint32_t m = min16(acc[v]);
            const bool lt = m < bY[qb];
            const bool eq = m == bY[qb];
            tie[qb] = lt ? 0u : (tie[qb] | (eq ? 1u : 0u));
            bT[qb] = lt ? t0 + v : bT[qb];
            bY[qb] = lt ? m : bY[qb];
        }
    }

    // all tiles of one LDS stage, pipelined across the two query blocks
    __device__ __forceinline__ void stage(const int8_t *lf, const int32_t *lh, uint32_t t0s,
                                          int lane, int grp) {
        constexpr int NS = ST / kTPS;
        v4i Af[kTPS][KB];
        v16i H[kTPS];
        v16i a0[kTPS], a1[kTPS];
        load_step(lf, lh, 0, lane, grp, Af, H);
        mma(0, Af, H, a0);
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const uint32_t t0 = t0s + (uint32_t)(u * kTPS);
            mma(1, Af, H, a1);
            track(0, a0, t0);
            if (u + 1 < NS) {
                load_step(lf, lh, u + 1, lane, grp, Af, H);
                mma(0, Af, H, a0);
            }
            track(1, a1, t0);
        }
    }
};

template <int DP, int ST>
__global__ __launch_bounds__(kBlock) void k_dense_rows(DevIndex ix, FrameBatch fb, Work w) {
    constexpr int KB = DP / 32;
    constexpr int STAGE = ST * KB * 1024;
    static_assert(ST % kTPS == 0, "tile pairs must divide a stage");
    __shared__ __attribute__((aligned(16))) int8_t s_f0[STAGE];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[STAGE];
    __shared__ __attribute__((aligned(16))) int32_t s_h0[ST * kTile];
    __shared__ __attribute__((aligned(16))) int32_t s_h1[ST * kTile];

    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t count = fb.all_full ? (uint32_t)fb.Q : w.counters[1];
    const uint32_t qbase = blockIdx.x * kBlockQ;
    if (qbase >= count) return;                   // whole block exits together

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int col = lane & 31, grp = lane >> 5;
    const int nstages = (int)(ix.n_pad / (kTile * ST));

    stage_dma<KB, ST>(ix.Rf, ix.Hf, 0, s_f0, s_h0, wv, lane);

    RowState<DP, ST> S;
    uint32_t qid[kQB];
    int qc[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                            grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) S.Bq[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
        qc[qb] = w.qc[qid[qb]];
        S.bY[qb] = ~0u;
        S.bT[qb] = 0;
        S.tie[qb] = 0;
    }
    __syncthreads();

    for (int sg = 0; sg < nstages; sg += 2) {
        if (sg + 1 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Hf, sg + 1, s_f1, s_h1, wv, lane);
        S.stage(s_f0, s_h0, (uint32_t)(sg * ST), lane, grp);
        __syncthreads();
        if (sg + 1 < nstages) {
            if (sg + 2 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Hf, sg + 2, s_f0, s_h0, wv, lane);
            S.stage(s_f1, s_h1, (uint32_t)((sg + 1) * ST), lane, grp);
            __syncthreads();
        }
    }

    // ---- merge the two lane groups (different rows of the same tiles)
    uint32_t Ym[kQB], Tm[kQB], Xm[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t oY = (uint32_t)__shfl_xor((int)S.bY[qb], 32, 64);
        const uint32_t oT = (uint32_t)__shfl_xor((int)S.bT[qb], 32, 64);
        const uint32_t oX = (uint32_t)__shfl_xor((int)S.tie[qb], 32, 64);
        const uint32_t y = S.bY[qb], t = S.bT[qb], x = S.tie[qb];
        Ym[qb] = min(y, oY);
        Tm[qb] = y < oY ? t : (oY < y ? oT : min(t, oT));
        Xm[qb] = y < oY ? x : (oY < y ? oX : (x | oX | (t != oT ? 1u : 0u)));
    }

    // ---- hand (Y, tile, tie) to the resolve kernel through the query's
    // record (records of dense-routed queries are free after the ring phase)
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const bool live = qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col) < count;
        if (live && grp == 0)
            w.rec[qid[qb]] = make_uint4(Ym[qb], (Tm[qb] << 1) | (Xm[qb] ? 1u : 0u), 0u, 0u);
    }
}

// One thread per dense query: recompute the 32 SSDs of the winning tile with
// v_dot4 and take the (SSD, index) minimum -- the global one, since every row
// outside that tile has a larger Y.  Queries flagged as ties go to the
// fallback list for the column-layout kernel.
template <int DP>
__global__ __launch_bounds__(256) void k_resolve(DevIndex ix, FrameBatch fb, Work w) {
    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t count = fb.all_full ? (uint32_t)fb.Q : w.counters[1];
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < count;
    const uint32_t q = live ? (list ? list[i] : i) : 0u;
    bool tie = false;
    if (live) {
        const uint4 rec = w.rec[q];
        tie = (rec.y & 1u) != 0;
        if (!tie) {
            const uint32_t T = rec.y >> 1;
            uint32_t a[DP / 4];
            const uint4 *src = reinterpret_cast<const uint4 *>(w.patches + (int64_t)q * DP);
#pragma unroll
            for (int k = 0; k < DP / 16; ++k) {
                const uint4 v = src[k];
                a[4 * k] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
            }
            const int Qc = w.qc[q];
            unsigned long long best = ~0ull;
            for (int m = 0; m < kTile; ++m) {
                const int64_t r = (int64_t)T * kTile + m;
                if (r >= ix.n) break;
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
            const FrameDesc *fdp = &fb.f[w.fid[q]];
            const int64_t ql = (int64_t)q - fdp->qbase;
            fdp->out[ql] = (int32_t)(uint32_t)best;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)(best >> 32);
        }
    }
    const unsigned long long tmask = __ballot(tie);
    if (tmask) {
        const int lane = threadIdx.x & 63;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&w.counters[2], (uint32_t)__popcll(tmask));
        base = __shfl(base, 0, 64);
        if (tie) {
            const unsigned lo = __builtin_amdgcn_mbcnt_lo((unsigned)tmask, 0u);
            w.fb_list[base + __builtin_amdgcn_mbcnt_hi((unsigned)(tmask >> 32), lo)] = q;
        }
    }
}

template <int DP>
hipError_t launch_rows_t(const DevIndex &ix, const FrameBatch &fb, const Work &w, hipStream_t st) {
    int64_t blocks = (fb.Q + kBlockQ - 1) / kBlockQ;
    if (blocks < 1) blocks = 1;
    constexpr int ST = DP <= 64 ? 8 : 4;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense_rows<DP, ST>), dim3((unsigned)blocks), dim3(kBlock),
                       0, st, ix, fb, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rb = (fb.Q + 255) / 256;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_resolve<DP>), dim3((unsigned)(rb < 1 ? 1 : rb)), dim3(256),
                       0, st, ix, fb, w);
    return hipGetLastError();
}

}  // namespace

bool dense_rows_supported(const DevIndex &ix) { return ix.Dp <= 96; }

hipError_t launch_dense_rows(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_rows_t<32>(ix, fb, w, st);
    case 64: return launch_rows_t<64>(ix, fb, w, st);
    case 96: return launch_rows_t<96>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
