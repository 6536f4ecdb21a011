// k_dense_rows.hip -- the row-layout dense search at the default block shape
// of every patch width (kernels in k_dense_rows.h), its k-NN variant, and the
// launch dispatch (other block shapes: k_dense_rows_shapes.hip).
#include "k_dense_rows.h"

namespace riann {

namespace {

// ---- k-NN over the class order (exact k nearest (SSD, index) pairs).
// The k nearest lie in the k tiles with the smallest (per-tile minimum Y,
// tile): for an element e of tile t, any k tiles ordered before t each hold
// an element strictly better than e (smaller Y; or the same Y in an earlier
// tile, hence the same or a smaller p, and at an equal SSD the same class and
// a lower index).  Each lane keeps the KN smallest (Y << TB) | tile keys of
// its lane group over the whole reference range (one key segment); the two
// groups' lists are merged into the KN smallest distinct tiles, all 32 rows
// of which the check recomputes exactly.

// ascending compare-exchange network on a bitonic sequence of N values
template <int N, typename T>
__device__ __forceinline__ void bitonic_clean(T (&v)[N]) {
#pragma unroll
    for (int d = N / 2; d >= 1; d /= 2)
#pragma unroll
        for (int i = 0; i < N; ++i)
            if ((i & d) == 0) {
                const T a = v[i], b = v[i + d];
                v[i] = a < b ? a : b;
                v[i + d] = a < b ? b : a;
            }
}

template <int DP, int ST, int KN>
__global__ __launch_bounds__(RowCfg<DP>::block) void k_dense_rows_knn(DevIndex ix, FrameBatch fb,
                                                                      Work w) {
    constexpr int KB = DP / 32, TB = row_tile_bits(DP);
    constexpr int kWaves = RowCfg<DP>::waves, kQB = KN >= 8 ? 2 : RowCfg<DP>::qb;
    constexpr int kWaveQ = 32 * kQB, kBlockQ = kWaveQ * kWaves;
    constexpr int STAGE = ST * KB * 1024;
    __shared__ __attribute__((aligned(16))) int8_t s_f0[STAGE];
    __shared__ __attribute__((aligned(16))) int8_t s_f1[STAGE];
    __shared__ __attribute__((aligned(16))) int32_t s_h0[ST * kTile];
    __shared__ __attribute__((aligned(16))) int32_t s_h1[ST * kTile];

    const uint32_t *list = fb.all_full ? nullptr : w.dense_list;
    const uint32_t count = fb.all_full ? (uint32_t)fb.Q : w.counters[1];
    const uint32_t qbase = blockIdx.x * kBlockQ;
    if (qbase >= count) return;                   // whole block exits together
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31, grp = lane >> 5;
    const int ns_all = (int)(ix.n_rows / (kTile * ST));
    stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, 0, s_f0, s_h0, wv, lane);

    RowState<DP, ST, kQB, KN> S;
    uint32_t qid[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        const uint32_t slot = min(qbase + (uint32_t)(wv * kWaveQ + qb * 32 + col), count - 1);
        qid[qb] = list ? list[slot] : slot;
        const int8_t *src = reinterpret_cast<const int8_t *>(w.patches) + (int64_t)qid[qb] * DP +
                            grp * 16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) S.Bq[qb][kb] = *reinterpret_cast<const v4i *>(src + kb * 32);
#pragma unroll
        for (int i = 0; i < KN; ++i) S.kl[qb][i] = ~0u;
    }
    __syncthreads();
    for (int sg = 0; sg < ns_all; sg += 2) {
        if (sg + 1 < ns_all) stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, sg + 1, s_f1, s_h1, wv, lane);
        S.template stage<ST>(s_f0, s_h0, (uint32_t)(sg * ST), lane, grp);
        __syncthreads();
        if (sg + 1 < ns_all) {
            if (sg + 2 < ns_all)
                stage_dma<KB, ST, kWaves>(ix.Rfr, ix.Hf, sg + 2, s_f0, s_h0, wv, lane);
            S.template stage<ST>(s_f1, s_h1, (uint32_t)((sg + 1) * ST), lane, grp);
            __syncthreads();
        }
    }

    // ---- the KN smallest distinct tiles of both lane groups (~0u: none):
    // the two sorted lists form a bitonic sequence; a key repeating an
    // earlier key's tile is dropped (that tile is already taken, at a
    // smaller Y), and the first KN remaining keys give the tiles
    constexpr uint32_t kTileMask = (1u << TB) - 1u;
    uint32_t tiles[kQB][KN];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        uint32_t v[2 * KN];
#pragma unroll
        for (int i = 0; i < KN; ++i) {
            const uint32_t o = (uint32_t)__shfl_xor((int)S.kl[qb][i], 32, 64);
            v[grp ? KN + i : i] = S.kl[qb][i];
            v[grp ? KN - 1 - i : 2 * KN - 1 - i] = o;
        }
        bitonic_clean<2 * KN>(v);
#pragma unroll
        for (int j = 0; j < KN; ++j) tiles[qb][j] = ~0u;
        uint32_t rank = 0;
#pragma unroll
        for (int i = 0; i < 2 * KN; ++i) {
            bool dup = v[i] == ~0u;
#pragma unroll
            for (int j = 0; j < i; ++j) dup = dup || ((v[j] & kTileMask) == (v[i] & kTileMask));
#pragma unroll
            for (int j = 0; j < KN; ++j)
                tiles[qb][j] = (!dup && rank == (uint32_t)j) ? (v[i] & kTileMask) : tiles[qb][j];
            rank += dup ? 0u : 1u;
        }
    }

    // ---- the check: 16 lanes per query, lane r taking rows r and r + 16 of
    // each tile; a lane-local sorted list of the KN smallest (SSD, index)
    // pairs, then a butterfly over the 16 lanes merging sorted lists (the
    // partner's list reversed makes a bitonic sequence whose KN smaller
    // halves are the merged KN smallest)
    const int sub = lane >> 4, r = lane & 15;
    const uint32_t wbase = qbase + (uint32_t)(wv * kWaveQ);
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
        for (int h = 0; h < 32; h += 4) {
            const int c = h + sub;
            const uint32_t q = (uint32_t)__shfl((int)qid[qb], c, 64);
            const bool live = wbase + (uint32_t)(qb * 32 + c) < count;
            unsigned long long L[KN];
            uint32_t tq[KN];                      // every lane takes part in the shuffles
#pragma unroll
            for (int i = 0; i < KN; ++i) {
                L[i] = ~0ull;
                tq[i] = (uint32_t)__shfl((int)tiles[qb][i], c, 64);
            }
            if (live) {
                uint4 a[DP / 16];
                const uint4 *pa = reinterpret_cast<const uint4 *>(w.patches + (int64_t)q * DP);
#pragma unroll
                for (int k = 0; k < DP / 16; ++k) a[k] = pa[k];
                const int qc = w.qc[q];
#pragma unroll
                for (int j = 0; j < KN; ++j) {
                    const uint32_t t = tq[j];
                    if (t == ~0u) continue;
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const int m = r + 16 * hh;
                        const int2 ri = ix.Rci[(int64_t)t * kTile + m];
                        if (ri.y < 0) continue;
                        uint4 u[DP / 16];
                        RowCheck<DP>::row_bytes(ix, t, m, u);
                        const uint32_t ssd = (uint32_t)(qc + ri.x + 2 * RowCheck<DP>::dot(a, u));
                        unsigned long long x = ((unsigned long long)ssd << 32) | (uint32_t)ri.y;
#pragma unroll
                        for (int i = 0; i < KN; ++i) {
                            const unsigned long long o = L[i];
                            L[i] = o < x ? o : x;
                            x = o < x ? x : o;
                        }
                    }
                }
            }
#pragma unroll
            for (int xm = 8; xm >= 1; xm >>= 1) {
                unsigned long long M[KN];
#pragma unroll
                for (int i = 0; i < KN; ++i) {
                    const unsigned long long pv = L[KN - 1 - i];
                    const unsigned lo = __shfl_xor((unsigned)pv, xm, 64);
                    const unsigned hi = __shfl_xor((unsigned)(pv >> 32), xm, 64);
                    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
                    M[i] = L[i] < o ? L[i] : o;
                }
                bitonic_clean<KN>(M);
#pragma unroll
                for (int i = 0; i < KN; ++i) L[i] = M[i];
            }
            if (live && r < fb.knn) {
                unsigned long long b = L[0];
#pragma unroll
                for (int i = 1; i < KN; ++i) b = r == i ? L[i] : b;
                const FrameDesc *fdp = &fb.f[w.fid[q]];
                const int64_t ql = (int64_t)q - fdp->qbase;
                fdp->out[ql * fb.knn + r] = (int32_t)(uint32_t)b;
                if (fdp->ssd) fdp->ssd[ql * fb.knn + r] = (uint32_t)(b >> 32);
            }
        }
    }
}

// Resolve step for the split chunks of a launch (the dense-list positions
// from whole * block_q on): 16 lanes per dense query take the lexicographic
// (Y, tile) minimum of the parts' records (disjoint tile ranges, so the first
// part reaching the smallest Y wins, with its group mask) and run the
// candidate check.  The records sit at the list position, so they load
// alongside the list.  A grid-stride loop whose trip count is uniform over
// the block; with no split chunk every block returns at once.

template <int DP, int KN>
hipError_t launch_rows_knn_kn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                              hipStream_t st) {
    constexpr int ST = DP <= 64 ? 8 : 4;
    constexpr int QB = KN >= 8 ? 2 : RowCfg<DP>::qb;
    constexpr int kBlockQ = 32 * QB * RowCfg<DP>::waves;
    const int64_t blocks = std::max<int64_t>(1, (fb.Q + kBlockQ - 1) / kBlockQ);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dense_rows_knn<DP, ST, KN>), dim3((unsigned)blocks),
                       dim3(RowCfg<DP>::block), 0, st, ix, fb, w);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_rows_knn_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             hipStream_t st) {
    if (fb.knn <= 2) return launch_rows_knn_kn<DP, 2>(ix, fb, w, st);
    if (fb.knn <= 4) return launch_rows_knn_kn<DP, 4>(ix, fb, w, st);
    return launch_rows_knn_kn<DP, 8>(ix, fb, w, st);
}

}  // namespace

bool dense_rows_supported(const DevIndex &ix) { return ix.n_rows > 0; }

bool dense_fused_supported(const DevIndex &ix) {
    return ix.n_rows > 0 && ix.Dp == 64 && ix.p == 8 && ix.C == 1;
}

bool knn_rows_supported(const DevIndex &ix) {
    return ix.n_rows > 0 && ix.n_rows / kTile <= ((int64_t)1 << row_tile_bits(ix.Dp));
}

hipError_t launch_dense_rows_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                 hipStream_t st) {
    if (fb.knn < 2 || fb.knn > kMaxKnn || !knn_rows_supported(ix)) return hipErrorInvalidValue;
    switch (ix.Dp) {
    case 32: return launch_rows_knn_t<32>(ix, fb, w, st);
    case 64: return launch_rows_knn_t<64>(ix, fb, w, st);
    case 96: return launch_rows_knn_t<96>(ix, fb, w, st);
    case 128: return launch_rows_knn_t<128>(ix, fb, w, st);
    case 160: return launch_rows_knn_t<160>(ix, fb, w, st);
    case 192: return launch_rows_knn_t<192>(ix, fb, w, st);
    case 224: return launch_rows_knn_t<224>(ix, fb, w, st);
    case 256: return launch_rows_knn_t<256>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense_rows(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             hipStream_t st) {
    if (ix.row_waves != 0 || ix.row_cols != 0) return launch_dense_rows_shape(ix, fb, w, st);
    switch (ix.Dp) {
    case 32: return launch_rows_t<32>(ix, fb, w, st);
    case 64: return launch_rows_t<64>(ix, fb, w, st);
    case 96: return launch_rows_t<96>(ix, fb, w, st);
    case 128: return launch_rows_t<128>(ix, fb, w, st);
    case 160: return launch_rows_t<160>(ix, fb, w, st);
    case 192: return launch_rows_t<192>(ix, fb, w, st);
    case 224: return launch_rows_t<224>(ix, fb, w, st);
    case 256: return launch_rows_t<256>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace riann
