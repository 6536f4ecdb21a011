// k_dense.hip -- exact exhaustive nearest-neighbour search on the int8
// matrix cores (v_mfma_i32_32x32x32_i8), used for full frames (first frame,
// scene cuts) and for queries routed away from the ring scan.
//
// With a = 127 - q and v = r - 128 (both int8), SSD(q, r) = Qc + Rc + 2<a, v>
// (encodings in riann_internal.h).  The GEMM gives acc = <a, v> exactly in
// int32.  For a fixed query, X = Rc + 2 acc + kBias = SSD - Qc + kBias lies in
// [0, 2^25), so the key (X << 6) | j -- j the tile's position inside a
// 64-tile segment -- orders (SSD, index) within one lane's column; it is
// formed with one v_lshl_add: key = ((Rc + kBias) << 6 | j) + (acc << 7).
// Each lane keeps a running unsigned minimum per query row; segment minima
// are merged into (X, index) with strict "<" (earlier = lower index), and a
// cross-lane reduction over the 32 columns finishes the argmin.
#include "riann_internal.h"

namespace riann {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;          // 4 wavefronts
constexpr int kWaveQ = 32;           // queries per wavefront (MFMA rows)
constexpr int kBlockQ = kWaveQ * (kBlock / 64);

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl_xor(lo, m, 64);
    hi = __shfl_xor(hi, m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// 16 bytes of a query patch starting at patch byte k0, each XOR-ed with
// 0x7F (a = 127 - q); bytes at k >= D are 0.
__device__ __forceinline__ v4i load_a16(const uint8_t *__restrict__ frame, int64_t pitch, int x,
                                        int y, int C, int rowlen, int D, int k0) {
    int dy = k0 / rowlen, rem = k0 - dy * rowlen;
    const uint8_t *row = frame + (int64_t)(y + dy) * pitch + (int64_t)x * C;
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = k0 + 4 * i + b;
            if (k < D) word |= ((uint32_t)row[rem] ^ 0x7Fu) << (8 * b);
            if (++rem == rowlen) { rem = 0; row += pitch; }
        }
        w[i] = word;
    }
    v4i r = {(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    return r;
}

template <int DP>
__global__ __launch_bounds__(kBlock) void k_dense(DevIndex ix, FrameArgs fa,
                                                   const uint32_t *__restrict__ list,
                                                   const uint32_t *__restrict__ count_dev,
                                                   uint32_t count_static,
                                                   int32_t *__restrict__ out,
                                                   uint32_t *__restrict__ ssd) {
    constexpr int KB = DP / 32;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 31, grp = lane >> 5;
    const uint32_t count = count_dev ? *count_dev : count_static;
    const int64_t ntiles = ix.n_pad / kTile;
    const int rowlen = ix.p * ix.C;

    for (uint32_t base = (blockIdx.x * (kBlock / 64) + wv) * kWaveQ; base < count;
         base += gridDim.x * kBlockQ) {
        // ---- A operand: query row `col` of this wavefront's 32 queries
        const uint32_t slot = min(base + (uint32_t)col, count - 1);
        const uint32_t qid = list ? list[slot] : slot;
        const int qi = (int)(qid / (uint32_t)fa.Wq), qj = (int)(qid % (uint32_t)fa.Wq);
        v4i A[KB];
        int s2 = 0, s1 = 0;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            A[kb] = load_a16(fa.frame, fa.pitch, qj * ix.s, qi * ix.s, ix.C, rowlen, ix.D,
                             kb * 32 + grp * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s2 = __builtin_amdgcn_sdot4(A[kb][e], A[kb][e], s2, false);
                s1 = __builtin_amdgcn_sdot4(A[kb][e], 0x01010101, s1, false);
            }
        }
        s2 += __shfl_xor(s2, 32, 64);
        s1 += __shfl_xor(s1, 32, 64);
        const int Qc_col = s2 + 2 * s1 + ix.D;   // Qc of query row `col`

        uint32_t best[16], gX[16], gI[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) { best[i] = ~0u; gX[i] = ~0u; gI[i] = ~0u; }

        const int8_t *rp = ix.Rv + (int64_t)col * DP + grp * 16;
        const int32_t *rc = ix.Rc + col;
        for (int64_t t = 0; t < ntiles; ++t) {
            v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const v4i B = *reinterpret_cast<const v4i *>(rp + kb * 32);
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[kb], B, acc, 0, 0, 0);
            }
            const uint32_t j = (uint32_t)(t & 63);
            const uint32_t rnj = ((uint32_t)rc[0] << 6) + (((uint32_t)kBias << 6) | j);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t key = rnj + ((uint32_t)acc[i] << 7);
                best[i] = min(best[i], key);
            }
            if (j == 63 || t == ntiles - 1) {
                const uint32_t seg = (uint32_t)(t >> 6);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint32_t X = best[i] >> 6;
                    const uint32_t idx = ((seg * 64u + (best[i] & 63u)) * kTile) + col;
                    if (X < gX[i]) { gX[i] = X; gI[i] = idx; }
                    best[i] = ~0u;
                }
            }
            rp += kTile * DP;
            rc += kTile;
        }
        // ---- cross-lane argmin over the 32 columns of each half-wavefront
        unsigned long long res = ~0ull;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            unsigned long long v = ((unsigned long long)gX[i] << 32) | gI[i];
#pragma unroll
            for (int m = 1; m < 32; m <<= 1) {
                unsigned long long o = shfl_xor_u64(v, m);
                v = o < v ? o : v;
            }
            if (col == i) res = v;   // lanes col < 16 keep row i = col
        }
        // accumulator register i of half `grp` holds row 8*(i/4) + 4*grp + i%4
        const int i = col;
        const int m = 8 * (i >> 2) + 4 * grp + (i & 3);
        const uint32_t qm = __shfl(qid, m, 64);
        const int Qc_m = __shfl(Qc_col, m, 64);
        if (col < 16 && base + (uint32_t)m < count) {
            const uint32_t X = (uint32_t)(res >> 32);
            out[qm] = (int32_t)(uint32_t)res;
            if (ssd) ssd[qm] = (uint32_t)((int)X - kBias + Qc_m);
        }
    }
}

template <int DP>
hipError_t launch_dense_t(const DevIndex &ix, const FrameArgs &fa, const uint32_t *list,
                          const uint32_t *count_dev, uint32_t count_static, int32_t *out,
                          uint32_t *ssd, hipStream_t st) {
    int64_t blocks = ((int64_t)count_static + kBlockQ - 1) / kBlockQ;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense<DP>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       ix, fa, list, count_dev, count_static, out, ssd);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(const DevIndex &ix, const FrameArgs &fa, const uint32_t *list,
                        const uint32_t *count_dev, uint32_t count_static, int32_t *out,
                        uint32_t *ssd, hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_dense_t<32>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 64: return launch_dense_t<64>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 96: return launch_dense_t<96>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 128: return launch_dense_t<128>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 160: return launch_dense_t<160>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 192: return launch_dense_t<192>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 224: return launch_dense_t<224>(ix, fa, list, count_dev, count_static, out, ssd, st);
    case 256: return launch_dense_t<256>(ix, fa, list, count_dev, count_static, out, ssd, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
