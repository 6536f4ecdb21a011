// k_recon.hip -- frame reconstruction from an ANN field (Sec. 4) and patch
// replacement with transformed references (Sec. 5).
//
// Every query patch (i, j) of a frame is replaced by appearance patch
// field[i][j] and overlapping patches are averaged.  A block owns a 64 x 16
// pixel tile: it stages the field entries of every patch touching the tile
// in LDS, then walks those patches row by row (consecutive threads on
// consecutive rows of one patch, so the appearance bytes arrive in whole
// cache lines) and adds each byte that lands in the tile into integer LDS
// accumulators; the coverage count of a pixel is a rectangle sum over a 2-D
// prefix sum of the valid field entries.  Integer sums do not depend
// on the order of the additions, so f_R = sum / count is exact to one float
// rounding and reproducible.  The normalised error
// E = ||gt - f_R|| / ||gt|| is reduced in fp64: per block into a partial,
// then one block adds the partials in index order, so the result does not
// depend on scheduling.
#include "riann_internal.h"

namespace riann {

namespace {

constexpr int kNT = 512;                            // threads per block
constexpr int kTX = 64, kTY = 16, kPY = kTY / (kNT / 64);   // tile; pixels per thread in y
constexpr int kBatch = 4;                           // patch rows whose loads are in flight
constexpr int kMaxFI = kTY + kMaxPatch, kMaxFJ = kTX + kMaxPatch;

__device__ __forceinline__ int ceil_div_nonneg(int a, int s) {   // ceil(a / s), a may be < 0
    return a <= 0 ? 0 : (a + s - 1) / s;
}

template <int CA>
__global__ __launch_bounds__(kNT) void k_recon(DevIndex ix, ReconArgs ra) {
    __shared__ int32_t s_f[kMaxFI * kMaxFJ];
    // accumulator rows padded by one word: the rows of one patch land in
    // different LDS banks
    constexpr int SROW = kTX * CA + 1;
    __shared__ uint32_t s_sum[kTY * SROW];
    __shared__ int32_t s_v[(kMaxFI + 1) * (kMaxFJ + 1)];   // valid-patch prefix sums
    __shared__ double s_red[3][kNT / 64];
    const int p = ix.p, s = ix.s;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY;
    // patches touching the tile: s*i <= y0 + kTY - 1 and s*i + p - 1 >= y0
    const int i_lo = ceil_div_nonneg(y0 - p + 1, s);
    const int i_hi = min(ra.Hq - 1, (y0 + kTY - 1) / s);
    const int j_lo = ceil_div_nonneg(x0 - p + 1, s);
    const int j_hi = min(ra.Wq - 1, (x0 + kTX - 1) / s);
    const int ni = i_hi - i_lo + 1, nj = j_hi - j_lo + 1;
    for (int k = threadIdx.x; k < ni * nj; k += kNT) {
        const int ii = k / nj, jj = k - ii * nj;
        s_f[ii * kMaxFJ + jj] = ra.field[(int64_t)(i_lo + ii) * ra.Wq + (j_lo + jj)];
    }
    for (int k = threadIdx.x; k < kTY * SROW; k += kNT) s_sum[k] = 0;
    __syncthreads();
    // coverage counts come from a 2-D prefix sum of the valid-patch mask:
    // s_v[(a) * (kMaxFJ + 1) + b] = number of valid entries in rows < a, cols < b
    constexpr int VJ = kMaxFJ + 1;
    if ((int)threadIdx.x <= ni) {                     // row prefix, one row per thread
        const int a = threadIdx.x;
        int run = 0;
        s_v[a * VJ] = 0;
        for (int b = 0; b < nj; ++b) {
            if (a > 0) {
                const int32_t r = s_f[(a - 1) * kMaxFJ + b];
                run += (r >= 0 && r < ix.n) ? 1 : 0;
            }
            s_v[a * VJ + b + 1] = run;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= nj) {                     // then column prefix
        const int b = threadIdx.x;
        for (int a = 1; a <= ni; ++a) s_v[a * VJ + b] += s_v[(a - 1) * VJ + b];
    }

    // ---- accumulate: one work item per (patch, patch row); consecutive
    // threads take consecutive rows of one patch, so their loads are adjacent
    const int rowlen = p * CA;                       // bytes of one patch row
    const uint8_t *base = ra.app ? ra.app : reinterpret_cast<const uint8_t *>(ix.Rv);
    const int64_t rowb = ra.app ? (int64_t)p * rowlen : (int64_t)ix.Dp;
    const uint32_t flip = ra.app ? 0u : 0x80u;       // the index stores r - 128
    const bool words = (rowlen % 4 == 0) && (rowb % 4 == 0) &&
                       ((reinterpret_cast<uintptr_t>(base) & 3u) == 0);
    const int items = ni * nj * p;
    // one patch row: its tile row (or -1 when it contributes nothing) and source
    auto locate = [&](int k, const uint8_t *&src, int &yy, int &xs) {
        yy = -1;
        src = base;
        xs = 0;
        if (k >= items) return;
        const int pi = k / p, dy = k - pi * p;
        const int ii = pi / nj, jj = pi - ii * nj;
        const int y = s * (i_lo + ii) + dy;
        if (y < y0 || y >= y0 + kTY) return;
        const int32_t r = s_f[ii * kMaxFJ + jj];
        if (r < 0 || r >= ix.n) return;              // not a reference: no patch
        xs = s * (j_lo + jj) - x0;                   // tile x of the patch's column 0
        src = base + (int64_t)r * rowb + (int64_t)dy * rowlen;
        yy = y - y0;
    };
    auto add_byte = [&](uint32_t *srow, int xs, int e, uint32_t v) {
        const int dx = e / CA, c = e - dx * CA;
        const int x = xs + dx;
        if (x >= 0 && x < kTX) atomicAdd(&srow[x * CA + c], v ^ flip);
    };
    if (words && rowlen <= 16) {
        // up to 4 words per row: the loads of kBatch rows are issued together
        const int nw = rowlen / 4;
        for (int k0 = threadIdx.x; k0 < items; k0 += kBatch * kNT) {
            const uint8_t *src[kBatch];
            int yy[kBatch], xs[kBatch];
            uint32_t wv4[kBatch][4];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                locate(k0 + u * kNT, src[u], yy[u], xs[u]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    wv4[u][q] = (yy[u] >= 0 && q < nw)
                                    ? reinterpret_cast<const uint32_t *>(src[u])[q] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (yy[u] < 0) continue;
                uint32_t *srow = s_sum + yy[u] * SROW;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q >= nw) break;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        add_byte(srow, xs[u], 4 * q + b, (wv4[u][q] >> (8 * b)) & 0xFFu);
                }
            }
        }
    } else {
        for (int k = threadIdx.x; k < items; k += kNT) {
            const uint8_t *src;
            int yy, xs;
            locate(k, src, yy, xs);
            if (yy < 0) continue;
            uint32_t *srow = s_sum + yy * SROW;
            for (int e = 0; e < rowlen; ++e) add_byte(srow, xs, e, src[e]);
        }
    }
    __syncthreads();

    // ---- write f_R = sum / count and the error sums
    const int x = x0 + (threadIdx.x & 63);
    double se = 0.0, sg = 0.0, nv = 0.0;
#pragma unroll
    for (int k = 0; k < kPY; ++k) {
        const int ty = (threadIdx.x >> 6) * kPY + k, y = y0 + ty;
        if (x >= ra.W || y >= ra.H) continue;
        // valid patches covering (y, x): window rows ia..ib, columns ja..jb
        const int ia = max(i_lo, ceil_div_nonneg(y - p + 1, s)) - i_lo, ib = min(i_hi, y / s) - i_lo;
        const int ja = max(j_lo, ceil_div_nonneg(x - p + 1, s)) - j_lo, jb = min(j_hi, x / s) - j_lo;
        uint32_t cnt = 0;
        if (ia <= ib && ja <= jb)
            cnt = (uint32_t)(s_v[(ib + 1) * VJ + jb + 1] - s_v[ia * VJ + jb + 1] -
                             s_v[(ib + 1) * VJ + ja] + s_v[ia * VJ + ja]);
        float *dst = ra.out + ((int64_t)y * ra.W + x) * CA;
#pragma unroll
        for (int c = 0; c < CA; ++c) {
            const uint32_t sm = s_sum[ty * SROW + (x - x0) * CA + c];
            const float fr = cnt ? (float)sm / (float)cnt : 0.0f;
            dst[c] = fr;
            if (ra.gt && cnt) {
                const double g = (double)ra.gt[(int64_t)y * ra.gt_pitch + (int64_t)x * CA + c];
                const double d = g - (double)fr;
                se += d * d;
                sg += g * g;
                nv += 1.0;
            }
        }
    }
    if (!ra.partials) return;
    // block reduction of the three sums, fixed order
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        se += __shfl_xor(se, m, 64);
        sg += __shfl_xor(sg, m, 64);
        nv += __shfl_xor(nv, m, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_red[0][wv] = se;
        s_red[1][wv] = sg;
        s_red[2][wv] = nv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *o = ra.partials + 3 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
        for (int q = 0; q < 3; ++q) {
            double a = 0.0;
            for (int k = 0; k < kNT / 64; ++k) a += s_red[q][k];
            o[q] = a;
        }
    }
}

// One block: adds the per-block partials in index order (thread t takes
// partials t, t + 256, ...; then a fixed tree) and writes {E, se, sg, values}.
__global__ __launch_bounds__(256) void k_recon_err(const double *partials, int64_t nb,
                                                    double *err) {
    __shared__ double s_r[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nb; b += 256)
        for (int q = 0; q < 3; ++q) a[q] += partials[3 * b + q];
    for (int q = 0; q < 3; ++q) s_r[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 3; ++q) s_r[q][threadIdx.x] += s_r[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double se = s_r[0][0], sg = s_r[1][0];
        err[0] = sg > 0.0 ? sqrt(se / sg) : 0.0;
        err[1] = se;
        err[2] = sg;
        err[3] = s_r[2][0];
    }
}

}  // namespace

int64_t recon_blocks(int H, int W) {
    return (int64_t)((W + kTX - 1) / kTX) * ((H + kTY - 1) / kTY);
}

hipError_t launch_recon(const DevIndex &ix, const ReconArgs &ra, double *err, hipStream_t st) {
    const dim3 grid((unsigned)((ra.W + kTX - 1) / kTX), (unsigned)((ra.H + kTY - 1) / kTY));
    switch (ra.Ca) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recon<1>), grid, dim3(kNT), 0, st, ix, ra); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recon<2>), grid, dim3(kNT), 0, st, ix, ra); break;
    case 3: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recon<3>), grid, dim3(kNT), 0, st, ix, ra); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_recon<4>), grid, dim3(kNT), 0, st, ix, ra); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ra.partials) return e;
    hipLaunchKernelGGL(k_recon_err, dim3(1), dim3(256), 0, st, (const double *)ra.partials,
                       (int64_t)grid.x * grid.y, err);
    return hipGetLastError();
}

}  // namespace riann
