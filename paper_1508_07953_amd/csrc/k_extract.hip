// k_extract.hip -- LDS-tiled patch extraction (the query patches q_{x,y,t}
// of one frame, every p x p x C window at stride s).
//
// A block owns a tile of 4 x 64 query positions of one frame of the launch's
// batch (tiles of all frames are numbered consecutively).  It copies the frame region
// those windows cover into LDS with coalesced byte loads (each frame byte is
// read from HBM once per tile and reused from LDS by up to (p/s)^2 windows),
// then each thread assembles one query's patch in (dy, dx, c) order, encodes
// every byte as a = q ^ 0x7F (127 - q as int8), pads it with zeros to Dp
// bytes and writes it as Dp/16 aligned 16-byte stores, plus
// Qc = sum over the D real bytes of (a + 1)^2.
#include "riann_internal.h"

namespace riann {

namespace {

constexpr int kTX = kExtTX, kTY = kExtTY;     // query columns x rows per block

template <int DP>
__global__ __launch_bounds__(kTX *kTY) void k_extract(DevIndex ix, FrameBatch fb, Work w) {
    extern __shared__ uint8_t s_tile[];
    const int p = ix.p, C = ix.C, s = ix.s, D = ix.D;
    // frame of this tile (tile ranges are consecutive per frame)
    int f = 0;
    while (f + 1 < fb.n && (int)blockIdx.x >= fb.f[f + 1].tbase) ++f;
    const FrameDesc &fa = fb.f[f];
    const int lt = (int)blockIdx.x - fa.tbase;
    const int tiles_x = (fa.Wq + kTX - 1) / kTX;
    const int qx0 = (lt % tiles_x) * kTX, qy0 = (lt / tiles_x) * kTY;
    const int nqx = min(kTX, fa.Wq - qx0), nqy = min(kTY, fa.Hq - qy0);
    // frame region covered by this block's windows
    const int rw = ((nqx - 1) * s + p) * C;     // bytes per region row
    const int rh = (nqy - 1) * s + p;
    const int ldw = ((kTX - 1) * s + p) * C;    // LDS row pitch (fixed)
    const uint8_t *src = fa.frame + (int64_t)(qy0 * s) * fa.pitch + (int64_t)(qx0 * s) * C;
    for (int e = threadIdx.x; e < rw * rh; e += kTX * kTY) {
        const int r = e / rw, cidx = e - r * rw;
        s_tile[r * ldw + cidx] = src[(int64_t)r * fa.pitch + cidx];
    }
    __syncthreads();

    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    if (tx >= nqx || ty >= nqy) return;
    const uint8_t *win = s_tile + (ty * s) * ldw + (tx * s) * C;
    const int rowlen = p * C;
    uint32_t wd[DP / 4];
    int dy = 0, rem = 0;
    int sa2 = 0, sa = 0;
#pragma unroll
    for (int i = 0; i < DP / 4; ++i) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 4 * i + b;
            const bool ok = k < D;
            const uint32_t v = ok ? ((uint32_t)win[dy * ldw + rem] ^ 0x7Fu) : 0u;
            word |= v << (8 * b);
            const bool wrap = rem + 1 == rowlen;
            rem = wrap ? 0 : rem + 1;
            dy = wrap ? dy + 1 : dy;
            if (dy >= p) dy = p - 1;             // k >= D: stay inside the window
        }
        wd[i] = word;
        sa2 = __builtin_amdgcn_sdot4((int)word, (int)word, sa2, false);
        sa = __builtin_amdgcn_sdot4((int)word, 0x01010101, sa, false);
    }
    const int64_t q = fa.qbase + (int64_t)(qy0 + ty) * fa.Wq + (qx0 + tx);
    uint4 *dst = reinterpret_cast<uint4 *>(w.patches + q * DP);
#pragma unroll
    for (int i = 0; i < DP / 16; ++i)
        dst[i] = make_uint4(wd[4 * i], wd[4 * i + 1], wd[4 * i + 2], wd[4 * i + 3]);
    // padding bytes are a = 0 and add nothing to the sums
    w.qc[q] = sa2 + 2 * sa + D;
    w.fid[q] = (uint8_t)f;
}

template <int DP>
hipError_t launch_extract_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                            hipStream_t st) {
    const size_t lds = (size_t)((kTY - 1) * ix.s + ix.p) * ((kTX - 1) * ix.s + ix.p) * ix.C;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract<DP>), dim3((unsigned)fb.ntiles),
                       dim3(kTX * kTY), lds, st, ix, fb, w);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_extract(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_extract_t<32>(ix, fb, w, st);
    case 64: return launch_extract_t<64>(ix, fb, w, st);
    case 96: return launch_extract_t<96>(ix, fb, w, st);
    case 128: return launch_extract_t<128>(ix, fb, w, st);
    case 160: return launch_extract_t<160>(ix, fb, w, st);
    case 192: return launch_extract_t<192>(ix, fb, w, st);
    case 224: return launch_extract_t<224>(ix, fb, w, st);
    case 256: return launch_extract_t<256>(ix, fb, w, st);
    default: return hipErrorInvalidValue;
    }
}

namespace {

// One thread per (pixel, byte of the stacked pixel): reads are contiguous per
// source frame row, writes contiguous in the output row.
__global__ __launch_bounds__(256) void k_stack(StackArgs sa) {
    const int TC = sa.T * sa.C;
    const int64_t row = (int64_t)sa.W * TC;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (k >= row) return;
    const int x = (int)(k / TC), tc = (int)(k - (int64_t)x * TC);
    const int t = tc / sa.C, c = tc - t * sa.C;
    sa.out[(int64_t)y * row + k] = sa.f[t][(int64_t)y * sa.pitch + (int64_t)x * sa.C + c];
}

}  // namespace

hipError_t launch_stack(const StackArgs &sa, hipStream_t st) {
    const int64_t row = (int64_t)sa.W * sa.T * sa.C;
    hipLaunchKernelGGL(k_stack, dim3((unsigned)((row + 255) / 256), (unsigned)sa.H), dim3(256), 0,
                       st, sa);
    return hipGetLastError();
}

}  // namespace riann
