// k_dense.hip -- exact exhaustive nearest-neighbour search on the int8
// matrix cores (v_mfma_i32_32x32x32_i8), used for whole frames (first frame,
// scene cuts) and for the queries the ring phase routes to it.
//
// With a = 127 - q and v = r - 128 (both int8), SSD(q, r) = Qc + Rc + 2<a, v>
// (encodings in riann_internal.h); the GEMM gives <a, v> exactly in int32.
// Work split: a block of 8 wavefronts owns 512 queries (64 per wavefront, as
// two 32-row MFMA A operands held in registers for the whole pass) and
// streams the reference set through LDS in stages of ST tiles x 32
// references.  The references are stored in MFMA fragment order, so a stage
// is a straight copy: each wavefront moves 1-KB chunks with global-to-LDS
// DMA (global_load_lds_dwordx4), no registers involved.  Two distinct LDS
// buffers alternate (the stage loop is unrolled by two so each buffer's role
// is static): the DMA of stage s+1 runs while stage s is computed, and the
// one barrier per stage both publishes the new stage and retires the old.
// Per tile each wavefront reads its B fragments from LDS (conflict-free, 16
// consecutive bytes per lane) and runs 2 x Dp/32 MFMAs.  Epilogue per
// (query, reference) pair: one v_lshl_add forms the key (X << jb | j) and a
// v_min3 (two tiles per step) keeps the running unsigned minimum per query
// row and lane column, which is the (SSD, index) argmin over that column.
// When the tile count exceeds the key's j range, tiles are processed in
// segments: at a segment end the winner's index is saved and the j bits of
// the running key are cleared, so an equal X in a later segment (a higher
// index) never displaces it.  A cross-lane reduction over the 32 columns
// finishes each query.
#include "riann_internal.h"

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

#ifndef RIANN_DENSE_WAVES
#define RIANN_DENSE_WAVES 8
#endif
#ifndef RIANN_DENSE_ST_NARROW
#define RIANN_DENSE_ST_NARROW 8     // tiles per LDS stage, Dp <= 64
#endif
#ifndef RIANN_DENSE_ST_WIDE
#define RIANN_DENSE_ST_WIDE 4       // tiles per LDS stage, Dp > 64
#endif
constexpr int kWaves = RIANN_DENSE_WAVES;   // wavefronts per block
constexpr int kBlock = 64 * kWaves;
constexpr int kQB = 2;                      // 32-query row blocks per wavefront
constexpr int kWaveQ = 32 * kQB;
constexpr int kBlockQ = kWaveQ * kWaves;
static_assert(kRefAlign % (kTile * RIANN_DENSE_ST_NARROW) == 0 &&
                  kRefAlign % (kTile * RIANN_DENSE_ST_WIDE) == 0,
              "reference padding must cover whole stages");

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl_xor(lo, m, 64);
    hi = __shfl_xor(hi, m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// DMA of stage `sg` (ST tiles of fragments plus their ST*32 key bases) into
// one LDS buffer.  Each 1-KB chunk is one wavefront-wide 16-byte-per-lane copy.
template <int KB, int ST>
__device__ __forceinline__ void stage_dma(const int8_t *__restrict__ gf,
                                          const uint32_t *__restrict__ gr, int sg, int8_t *lf,
                                          uint32_t *lr, int wv, int lane) {
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
        __builtin_amdgcn_global_load_lds((glb_void *)(gr + (int64_t)sg * ST * kTile + lane * 4),
                                         (lds_void *)lr, 16, 0, 0);
}

template <int DP, bool SEG, int TPS, int ST>
struct DenseState {
    static constexpr int KB = DP / 32;
    v4i A[kQB][KB];
    uint32_t best[kQB][16];
    uint32_t gI[SEG ? kQB : 1][16];
    uint32_t segbase;

    // B fragments and key bases of step u (TPS tiles) of an LDS stage
    __device__ __forceinline__ void load_step(const int8_t *lf, const uint32_t *lr, int u,
                                              int lane, int col, uint32_t j0, v4i (&B)[TPS][KB],
                                              uint32_t (&rnj)[TPS]) {
#pragma unroll
        for (int v = 0; v < TPS; ++v) {
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                B[v][kb] = *reinterpret_cast<const v4i *>(lf + ((u * TPS + v) * KB + kb) * 1024 +
                                                          lane * 16);
            rnj[v] = lr[(u * TPS + v) * kTile + col] | (j0 + v);
        }
    }

    __device__ __forceinline__ void mma(int qb, const v4i (&B)[TPS][KB], v16i (&acc)[TPS]) {
#pragma unroll
        for (int v = 0; v < TPS; ++v) {
            acc[v] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                acc[v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[qb][kb], B[v][kb], acc[v], 0, 0,
                                                               0);
        }
    }

    __device__ __forceinline__ void epilogue(int qb, const v16i (&acc)[TPS],
                                             const uint32_t (&rnj)[TPS], uint32_t ash) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t m = best[qb][i];
#pragma unroll
            for (int v = 0; v < TPS; ++v) m = min(m, rnj[v] + ((uint32_t)acc[v][i] << ash));
            best[qb][i] = m;
        }
    }

    // All tiles of one LDS stage (tile t0s = sg * ST is its first), software
    // pipelined across the two query blocks: the MFMAs of block 1 run while
    // block 0's epilogue executes, and those of block 0 for the next step
    // while block 1's epilogue executes.
    __device__ __forceinline__ void stage(const int8_t *lf, const uint32_t *lr, uint32_t t0s,
                                          int lane, int col, uint32_t jb, uint32_t ash,
                                          uint32_t seglen, int64_t ntiles) {
        constexpr int NS = ST / TPS;
        v4i Bc[TPS][KB], Bn[TPS][KB];
        uint32_t rc[TPS], rn[TPS];
        v16i a0[TPS], a1[TPS];
        uint32_t j0 = SEG ? (t0s - segbase + 1) : t0s;
        load_step(lf, lr, 0, lane, col, j0, Bc, rc);
        mma(0, Bc, a0);
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const uint32_t t0 = t0s + (uint32_t)(u * TPS);
            mma(1, Bc, a1);
            epilogue(0, a0, rc, ash);
            const bool seg_end = SEG && (j0 + TPS - 1 == seglen || (int64_t)t0 + TPS == ntiles);
            const uint32_t jn = seg_end ? 1u : j0 + TPS;
            if (u + 1 < NS) {
                load_step(lf, lr, u + 1, lane, col, SEG ? jn : t0 + TPS, Bn, rn);
                mma(0, Bn, a0);
            }
            epilogue(1, a1, rc, ash);
            if (seg_end) {
                const uint32_t jm = (1u << jb) - 1;
#pragma unroll
                for (int qb = 0; qb < (SEG ? kQB : 1); ++qb)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const uint32_t jj = best[qb][i] & jm;
                        if (jj) {
                            gI[qb][i] = (segbase + jj - 1) * kTile + col;
                            best[qb][i] &= ~jm;
                        }
                    }
                segbase = t0 + TPS;
            }
            if (u + 1 < NS) {
#pragma unroll
                for (int v = 0; v < TPS; ++v) {
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb) Bc[v][kb] = Bn[v][kb];
                    rc[v] = rn[v];
                }
                j0 = SEG ? jn : t0 + TPS;
            }
        }
    }
};

template <int DP, bool SEG, int TPS, int ST>
__global__ __launch_bounds__(kBlock) void k_dense(DevIndex ix, FrameBatch fb, Work w,
                                                   const uint32_t *__restrict__ list,
                                                   const uint32_t *__restrict__ count_ptr) {
    constexpr int KB = DP / 32;
    constexpr int STAGE = ST * KB * 1024;         // fragment bytes of one stage
    static_assert(ST % TPS == 0, "tiles per step must divide a stage");
    __shared__ __attribute__((aligned(16))) int8_t s_f0[STAGE];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[STAGE];
    __shared__ __attribute__((aligned(16))) uint32_t s_r0[ST * kTile];
    __shared__ __attribute__((aligned(16))) uint32_t s_r1[ST * kTile];

    // no list: every query of the batch; otherwise the list and its count
    const uint32_t count = list ? *count_ptr : (uint32_t)fb.Q;
    const uint32_t qbase = blockIdx.x * kBlockQ;
    if (qbase >= count) return;                   // whole block exits together

    // the wavefront index is uniform: keep it (and the DMA addresses) in SGPRs
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31, grp = lane >> 5;
    const int nstages = (int)(ix.n_pad / (kTile * ST));
    const int64_t ntiles = ix.n_pad / kTile;
    const uint32_t jb = (uint32_t)ix.jb, ash = jb + 1;
    // SEG: j runs 1..seglen, seglen a multiple of TPS, so a segment always
    // ends on the last tile of a step (segments start on step boundaries)
    const uint32_t seglen = (1u << jb) - TPS;

    // stage 0 DMA first, so it overlaps the query loads
    stage_dma<KB, ST>(ix.Rf, ix.Rk, 0, s_f0, s_r0, wv, lane);

    // ---- A operands: rows `col` of the wavefront's two 32-query blocks,
    // 16 aligned bytes per k-block from the extracted patches
    DenseState<DP, SEG, TPS, ST> S;
    uint32_t qid[kQB];
    int qc[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                            grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) S.A[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
        qc[qb] = w.qc[qid[qb]];
    }
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            S.best[qb][i] = ~0u;
            S.gI[SEG ? qb : 0][i] = 0;
        }
    S.segbase = 0;
    __syncthreads();

    for (int sg = 0; sg < nstages; sg += 2) {
        if (sg + 1 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Rk, sg + 1, s_f1, s_r1, wv, lane);
        S.stage(s_f0, s_r0, (uint32_t)(sg * ST), lane, col, jb, ash, seglen, ntiles);
        __syncthreads();
        if (sg + 1 < nstages) {
            if (sg + 2 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Rk, sg + 2, s_f0, s_r0, wv, lane);
            S.stage(s_f1, s_r1, (uint32_t)((sg + 1) * ST), lane, col, jb, ash, seglen, ntiles);
            __syncthreads();
        }
    }

    // ---- per 32-query block: transpose-reduce over the 32 columns.  Four
    // butterfly steps (half = 8, 4, 2, 1) leave lane `col` with the minimum of
    // register i = col & 15 over the 16 columns that share bit 4 of `col`; a
    // final exchange with col ^ 16 completes it.  Lanes with col >> 4 == qb
    // then write row 8*(i/4) + 4*grp + i%4 of block qb.
    const uint32_t jm = (1u << jb) - 1;
    const int i_own = col & 15;
    const int m_own = 8 * (i_own >> 2) + 4 * grp + (i_own & 3);
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        unsigned long long v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t b = S.best[qb][i];
            const uint32_t idx = SEG ? S.gI[SEG ? qb : 0][i] : (b & jm) * kTile + col;
            v[i] = ((unsigned long long)(b >> jb) << 32) | idx;
        }
#pragma unroll
        for (int half = 8; half >= 1; half >>= 1) {
            const bool up = (col & half) != 0;
#pragma unroll
            for (int r = 0; r < half; ++r) {
                const unsigned long long keep = up ? v[r + half] : v[r];
                const unsigned long long send = up ? v[r] : v[r + half];
                const unsigned long long got = shfl_xor_u64(send, half);
                v[r] = got < keep ? got : keep;
            }
        }
        const unsigned long long other = shfl_xor_u64(v[0], 16);
        const unsigned long long res = other < v[0] ? other : v[0];
        const uint32_t qm = __shfl(qid[qb], m_own, 64);
        const int Qc_m = __shfl(qc[qb], m_own, 64);
        if ((col >> 4) == qb && qbase + (uint32_t)(wv * kWaveQ + qb * 32 + m_own) < count) {
            const uint32_t X = (uint32_t)(res >> 32);
            const FrameDesc *fdp = &fb.f[w.fid[qm]];
            const int64_t ql = (int64_t)qm - fdp->qbase;
            fdp->out[ql] = (int32_t)(uint32_t)res;
            if (fdp->ssd) fdp->ssd[ql] = (uint32_t)((int)X - ix.bias + Qc_m);
        }
    }
}

// ---------------------------------------------------------------- k-NN
// Dense k-NN search (column layout, unsegmented keys): each wavefront holds
// 32 queries as one MFMA A operand; lane (col, group) keeps, for each of its
// 16 query rows, the KN smallest keys (X << jb | tile) of its reference column
// in a sorted register list (one v_min and one v_max per level).  At the end,
// KN rounds of a 32-lane minimum over the list heads of each row, on
// (X, index) pairs, give the row's KN nearest in ascending order (KN = 2, 4
// or 8; the first k are written).
template <int DP, int KN, int ST>
__global__ __launch_bounds__(kBlock) void k_dense_knn(DevIndex ix, FrameBatch fb, Work w,
                                                       const uint32_t *__restrict__ list,
                                                       const uint32_t *__restrict__ count_ptr) {
    constexpr int KB = DP / 32;
    constexpr int STAGE = ST * KB * 1024;
    constexpr int BQ = 32 * kWaves;               // queries per block
    __shared__ __attribute__((aligned(16))) int8_t s_f0[STAGE];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[STAGE];
    __shared__ __attribute__((aligned(16))) uint32_t s_r0[ST * kTile];
    __shared__ __attribute__((aligned(16))) uint32_t s_r1[ST * kTile];

    const uint32_t count = list ? *count_ptr : (uint32_t)fb.Q;
    const uint32_t qbase = blockIdx.x * BQ;
    if (qbase >= count) return;                   // whole block exits together
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31, grp = lane >> 5;
    const int nstages = (int)(ix.n_pad / (kTile * ST));
    const uint32_t jb = (uint32_t)ix.jb, ash = jb + 1;

    stage_dma<KB, ST>(ix.Rf, ix.Rk, 0, s_f0, s_r0, wv, lane);
    const uint32_t slot = min(qbase + (uint32_t)(wv * 32 + col), count - 1);
    const uint32_t qid = list ? list[slot] : slot;
    v4i A[KB];
    {
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid * DP + grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) A[kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
    }
    const int qc = w.qc[qid];
    uint32_t lst[16][KN];
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
        for (int q = 0; q < KN; ++q) lst[i][q] = ~0u;
    __syncthreads();

    auto tile = [&](const int8_t *lf, const uint32_t *lr, int u, uint32_t t) {
        v4i B[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            B[kb] = *reinterpret_cast<const v4i *>(lf + (u * KB + kb) * 1024 + lane * 16);
        const uint32_t rnj = lr[u * kTile + col] | t;
        v16i acc = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[kb], B[kb], acc, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t v = rnj + ((uint32_t)acc[i] << ash);
#pragma unroll
            for (int q = 0; q < KN; ++q) {        // sorted insertion
                const uint32_t o = lst[i][q];
                lst[i][q] = min(o, v);
                v = max(o, v);
            }
        }
    };
    for (int sg = 0; sg < nstages; sg += 2) {
        if (sg + 1 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Rk, sg + 1, s_f1, s_r1, wv, lane);
#pragma unroll
        for (int u = 0; u < ST; ++u) tile(s_f0, s_r0, u, (uint32_t)(sg * ST + u));
        __syncthreads();
        if (sg + 1 < nstages) {
            if (sg + 2 < nstages) stage_dma<KB, ST>(ix.Rf, ix.Rk, sg + 2, s_f0, s_r0, wv, lane);
#pragma unroll
            for (int u = 0; u < ST; ++u) tile(s_f1, s_r1, u, (uint32_t)((sg + 1) * ST + u));
            __syncthreads();
        }
    }

    // ---- merge the 32 columns of every query row
    const uint32_t jm = (1u << jb) - 1;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = 8 * (i >> 2) + 4 * grp + (i & 3);   // the row register i holds
        const uint32_t qm = (uint32_t)__shfl((int)qid, m, 64);
        const int Qc_m = __shfl(qc, m, 64);
        const bool live = qbase + (uint32_t)(wv * 32 + m) < count;
        const FrameDesc *fdp = &fb.f[w.fid[qm]];
        const int64_t ql = (int64_t)qm - fdp->qbase;
#pragma unroll
        for (int r = 0; r < KN; ++r) {
            const uint32_t h = lst[i][0];
            const unsigned long long mine =
                ((unsigned long long)(h >> jb) << 32) | ((h & jm) * kTile + (uint32_t)col);
            unsigned long long b = mine;
#pragma unroll
            for (int x = 16; x >= 1; x >>= 1) {
                const unsigned lo = __shfl_xor((unsigned)b, x, 64);
                const unsigned hi = __shfl_xor((unsigned)(b >> 32), x, 64);
                const unsigned long long o = ((unsigned long long)hi << 32) | lo;
                b = o < b ? o : b;
            }
            if (mine == b) {                             // the one column holding it pops
#pragma unroll
                for (int q = 0; q + 1 < KN; ++q) lst[i][q] = lst[i][q + 1];
                lst[i][KN - 1] = ~0u;
            }
            if (col == 0 && live && r < fb.knn) {
                fdp->out[ql * fb.knn + r] = (int32_t)(uint32_t)b;
                if (fdp->ssd)
                    fdp->ssd[ql * fb.knn + r] =
                        (uint32_t)((int)(uint32_t)(b >> 32) - ix.bias + Qc_m);
            }
        }
    }
}

template <int DP, int KN>
hipError_t launch_knn_t2(const DevIndex &ix, const FrameBatch &fb, const Work &w, hipStream_t st) {
    constexpr int ST = DP <= 64 ? 8 : 4;
    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t *count = fb.all_full ? nullptr : w.counters + 1;
    int64_t blocks = (fb.Q + 32 * kWaves - 1) / (32 * kWaves);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense_knn<DP, KN, ST>), dim3((unsigned)blocks),
                       dim3(kBlock), 0, st, ix, fb, w, list, count);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_knn_t(const DevIndex &ix, const FrameBatch &fb, const Work &w, hipStream_t st) {
    // lists of 2, 4 or 8 entries; the first fb.knn of them are written
    if (fb.knn < 2 || fb.knn > kMaxKnn) return hipErrorInvalidValue;
    if (fb.knn <= 2) return launch_knn_t2<DP, 2>(ix, fb, w, st);
    if (fb.knn <= 4) return launch_knn_t2<DP, 4>(ix, fb, w, st);
    return launch_knn_t2<DP, 8>(ix, fb, w, st);
}

template <int DP>
hipError_t launch_dense_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          const uint32_t *list, const uint32_t *count, hipStream_t st) {
    int64_t blocks = (fb.Q + kBlockQ - 1) / kBlockQ;
    if (blocks < 1) blocks = 1;
    // tile pairs (one v_min3 per update) while the epilogue is the bound,
    // single tiles for wide patches, where the matrix cores are; 8-tile
    // stages while they fit two blocks per CU in LDS
    constexpr int TPS = DP <= 96 ? 2 : 1;
    constexpr int ST = DP <= 64 ? RIANN_DENSE_ST_NARROW : RIANN_DENSE_ST_WIDE;
    const bool seg = (ix.n_pad / kTile) > (int64_t)(1u << ix.jb);
    if (seg)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense<DP, true, TPS, ST>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, ix, fb, w, list, count);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense<DP, false, TPS, ST>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, ix, fb, w, list, count);
    return hipGetLastError();
}

hipError_t dispatch(const DevIndex &ix, const FrameBatch &fb, const Work &w, const uint32_t *list,
                    const uint32_t *count, hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_dense_t<32>(ix, fb, w, list, count, st);
    case 64: return launch_dense_t<64>(ix, fb, w, list, count, st);
    case 96: return launch_dense_t<96>(ix, fb, w, list, count, st);
    case 128: return launch_dense_t<128>(ix, fb, w, list, count, st);
    case 160: return launch_dense_t<160>(ix, fb, w, list, count, st);
    case 192: return launch_dense_t<192>(ix, fb, w, list, count, st);
    case 224: return launch_dense_t<224>(ix, fb, w, list, count, st);
    case 256: return launch_dense_t<256>(ix, fb, w, list, count, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_dense(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                        hipStream_t st) {
    return fb.all_full ? dispatch(ix, fb, w, nullptr, nullptr, st)
                       : dispatch(ix, fb, w, w.dense_list, w.counters + 1, st);
}

bool knn_dense_supported(const DevIndex &ix) {
    return (ix.n_pad / kTile) <= ((int64_t)1 << ix.jb);
}

hipError_t launch_dense_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                            hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_knn_t<32>(ix, fb, w, st);
    case 64: return launch_knn_t<64>(ix, fb, w, st);
    case 96: return launch_knn_t<96>(ix, fb, w, st);
    case 128: return launch_knn_t<128>(ix, fb, w, st);
    case 160: return launch_knn_t<160>(ix, fb, w, st);
    case 192: return launch_knn_t<192>(ix, fb, w, st);
    case 224: return launch_knn_t<224>(ix, fb, w, st);
    case 256: return launch_knn_t<256>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense_list(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             const uint32_t *list, const uint32_t *count, hipStream_t st) {
    return dispatch(ix, fb, w, list, count, st);
}

}  // namespace riann
