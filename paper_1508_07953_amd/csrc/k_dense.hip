// k_dense.hip -- exact exhaustive nearest-neighbour search on the int8
// matrix cores (v_mfma_i32_32x32x32_i8), used for whole frames (first frame,
// scene cuts) and for the queries the ring phase routes to it.
//
// With a = 127 - q and v = r - 128 (both int8), SSD(q, r) = Qc + Rc + 2<a, v>
// (encodings in riann_internal.h); the GEMM gives <a, v> exactly in int32.
// Work split: a block of 4 wavefronts owns 256 queries (64 per wavefront, as
// two 32-row MFMA A operands held in registers for the whole pass) and
// streams the reference set through LDS in stages of 4 tiles x 32 references,
// double buffered; the stage copy is a straight coalesced copy because the
// references are stored in MFMA fragment order.  Per tile each wavefront
// reads its B fragments from LDS (conflict-free, 16 consecutive bytes per
// lane) and runs 2 x Dp/32 MFMAs.  Epilogue per (query, reference) pair: one
// v_lshl_add forms the key (X << jb | j) and a v_min3 keeps the running
// unsigned minimum per query row and lane column, which is the (SSD, index)
// argmin over that column.  When the tile count exceeds the key's j range,
// tiles are processed in segments: at a segment end the winner's index is
// saved and the j bits of the running key are cleared, so an equal X in a
// later segment (a higher index) never displaces it.  A cross-lane
// reduction over the 32 columns finishes each query.
#include "riann_internal.h"

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;                 // 4 wavefronts
constexpr int kQB = 2;                      // 32-query row blocks per wavefront
constexpr int kWaveQ = 32 * kQB;
constexpr int kBlockQ = kWaveQ * (kBlock / 64);

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl_xor(lo, m, 64);
    hi = __shfl_xor(hi, m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

template <int DP, bool SEG, int TPS>
__global__ __launch_bounds__(kBlock) void k_dense(DevIndex ix, Work w,
                                                   const uint32_t *__restrict__ list,
                                                   const uint32_t *__restrict__ count_dev,
                                                   uint32_t count_static,
                                                   int32_t *__restrict__ out,
                                                   uint32_t *__restrict__ ssd) {
    constexpr int KB = DP / 32;
    constexpr int FRAG = KB * 1024;               // fragment bytes of one tile
    constexpr int STAGE = kStageTiles * FRAG;     // fragment bytes of one stage
    constexpr int PIECES = STAGE / 16 / kBlock;   // 16-byte copies per thread
    static_assert(PIECES * 16 * kBlock == STAGE, "stage copy must divide evenly");
    static_assert(kStageTiles % TPS == 0, "tiles per step must divide a stage");
    __shared__ __attribute__((aligned(16))) int8_t s_frag[2][STAGE];
    __shared__ __attribute__((aligned(16))) uint32_t s_rk[2][kStageTiles * kTile];

    const uint32_t count = count_dev ? *count_dev : count_static;
    const uint32_t qbase = blockIdx.x * kBlockQ;
    if (qbase >= count) return;                   // whole block exits together

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int col = lane & 31, grp = lane >> 5;
    const int nstages = (int)(ix.n_pad / (kTile * kStageTiles));
    const uint32_t jb = (uint32_t)ix.jb, ash = jb + 1;
    // SEG: j runs 1..seglen, seglen a multiple of TPS, so a segment always
    // ends on the last tile of a step (segments start on step boundaries)
    const uint32_t seglen = (1u << jb) - TPS;
    const uint4 *gfrag = reinterpret_cast<const uint4 *>(ix.Rf);
    const uint4 *grk = reinterpret_cast<const uint4 *>(ix.Rk);

    // ---- stage 0 copy first, so its latency overlaps the query loads
#pragma unroll
    for (int k = 0; k < PIECES; ++k)
        reinterpret_cast<uint4 *>(s_frag[0])[tid + k * kBlock] = gfrag[tid + k * kBlock];
    if (tid < kStageTiles * kTile / 4) reinterpret_cast<uint4 *>(s_rk[0])[tid] = grk[tid];

    // ---- A operands: rows `col` of the wavefront's two 32-query blocks,
    // 16 aligned bytes per k-block from the extracted patches
    v4i A[kQB][KB];
    uint32_t qid[kQB];
    int qc[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                            grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) A[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
        qc[qb] = w.qc[qid[qb]];
    }

    uint32_t best[kQB][16];
    uint32_t gI[SEG ? kQB : 1][16];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
        for (int i = 0; i < 16; ++i) best[qb][i] = ~0u;
    if (SEG) {
#pragma unroll
        for (int qb = 0; qb < (SEG ? kQB : 1); ++qb)
#pragma unroll
            for (int i = 0; i < 16; ++i) gI[qb][i] = 0;
    }
    __syncthreads();

    uint32_t segbase = 0;   // first tile of the current segment (SEG)
    for (int sg = 0; sg < nstages; ++sg) {
        const int buf = sg & 1;
        const bool more = sg + 1 < nstages;
        // prefetch the next stage into registers (the last stage re-reads
        // itself, harmlessly, so the loads are unconditional)
        const int nx = more ? sg + 1 : sg;
        uint4 pf[PIECES];
        const uint4 *src = gfrag + (int64_t)nx * (STAGE / 16);
#pragma unroll
        for (int k = 0; k < PIECES; ++k) pf[k] = src[tid + k * kBlock];
        const uint4 pr = grk[(int64_t)nx * (kStageTiles * kTile / 4) + (tid & 31)];
#pragma unroll 1
        for (int tp = 0; tp < kStageTiles; tp += TPS) {
            // TPS tiles per step: with two, each best[] update is one v_min3
            const uint32_t t0 = (uint32_t)(sg * kStageTiles + tp);
            const uint32_t j0 = SEG ? (t0 - segbase + 1) : t0;
            v4i B[TPS][KB];
            uint32_t rnj[TPS];
#pragma unroll
            for (int u = 0; u < TPS; ++u) {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    B[u][kb] = *reinterpret_cast<const v4i *>(
                        &s_frag[buf][((tp + u) * KB + kb) * 1024 + lane * 16]);
                rnj[u] = s_rk[buf][(tp + u) * kTile + col] | (j0 + u);
            }
#pragma unroll
            for (int qb = 0; qb < kQB; ++qb) {
                v16i acc[TPS];
#pragma unroll
                for (int u = 0; u < TPS; ++u) {
                    acc[u] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        acc[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[qb][kb], B[u][kb],
                                                                       acc[u], 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    uint32_t m = best[qb][i];
#pragma unroll
                    for (int u = 0; u < TPS; ++u)
                        m = min(m, rnj[u] + ((uint32_t)acc[u][i] << ash));
                    best[qb][i] = m;
                }
            }
            if (SEG && (j0 + TPS - 1 == seglen || (int64_t)t0 + TPS == ix.n_pad / kTile)) {
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
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < PIECES; ++k)
                reinterpret_cast<uint4 *>(s_frag[buf ^ 1])[tid + k * kBlock] = pf[k];
            if (tid < kStageTiles * kTile / 4) reinterpret_cast<uint4 *>(s_rk[buf ^ 1])[tid] = pr;
        }
        __syncthreads();
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
            const uint32_t b = best[qb][i];
            const uint32_t idx = SEG ? gI[SEG ? qb : 0][i] : (b & jm) * kTile + col;
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
            out[qm] = (int32_t)(uint32_t)res;
            if (ssd) ssd[qm] = (uint32_t)((int)X - ix.bias + Qc_m);
        }
    }
}

template <int DP>
hipError_t launch_dense_t(const DevIndex &ix, const Work &w, const uint32_t *list,
                          const uint32_t *count_dev, uint32_t count_static, int32_t *out,
                          uint32_t *ssd, hipStream_t st) {
    int64_t blocks = ((int64_t)count_static + kBlockQ - 1) / kBlockQ;
    if (blocks < 1) blocks = 1;
    // tile pairs (one v_min3 per update) while the epilogue is the bound;
    // single tiles for wide patches, where the matrix cores are
    constexpr int TPS = DP <= 96 ? 2 : 1;
    const bool seg = (ix.n_pad / kTile) > (int64_t)(1u << ix.jb);
    if (seg)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense<DP, true, TPS>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, ix, w, list, count_dev, count_static, out, ssd);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense<DP, false, TPS>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, ix, w, list, count_dev, count_static, out, ssd);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(const DevIndex &ix, const Work &w, const uint32_t *list,
                        const uint32_t *count_dev, uint32_t count_static, int32_t *out,
                        uint32_t *ssd, hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_dense_t<32>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 64: return launch_dense_t<64>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 96: return launch_dense_t<96>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 128: return launch_dense_t<128>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 160: return launch_dense_t<160>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 192: return launch_dense_t<192>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 224: return launch_dense_t<224>(ix, w, list, count_dev, count_static, out, ssd, st);
    case 256: return launch_dense_t<256>(ix, w, list, count_dev, count_static, out, ssd, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
