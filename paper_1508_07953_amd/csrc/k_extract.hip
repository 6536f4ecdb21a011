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
// Qc = sum over the D real bytes of (a + 1)^2.  When a window row holds a
// whole number of 32-bit words (p*C % 4 == 0: 8x8 gray, 8x8x3, 12x12, ...)
// a template instance reads each row as aligned LDS words and funnel-shifts
// them into place (v_alignbyte); other shapes assemble byte by byte.  Block 0
// also clears the launch's ring and dense list counters, which the ring
// kernel after it fills.
#include "riann_internal.h"

namespace riann {

namespace {

constexpr int kTX = kExtTX, kTY = kExtTY;     // query columns x rows per block

// LDS row pitch of a tile's frame region: its widest row, rounded up to
// whole words; ext_lds_bytes adds one spare word (see k_extract_rows).
__host__ __device__ __forceinline__ int ext_ldw(int p, int C, int s) {
    return ((((kTX - 1) * s + p) * C) + 3) & ~3;
}
__host__ __device__ __forceinline__ size_t ext_lds_bytes(int p, int C, int s) {
    return (size_t)((kTY - 1) * s + p) * ext_ldw(p, C, s) + 4;
}

// The block's tile: its frame, first query position and extent, and the
// frame region its windows cover, copied into LDS (row pitch ldw).
struct ExtTile {
    int f, qx0, qy0, nqx, nqy, ldw;
    const FrameDesc *fa;
};

__device__ __forceinline__ ExtTile load_tile(const DevIndex &ix, const FrameBatch &fb,
                                             uint8_t *s_tile) {
    const int p = ix.p, C = ix.C, s = ix.s;
    ExtTile t;
    // frame of this tile (tile ranges are consecutive per frame)
    t.f = 0;
    while (t.f + 1 < fb.n && (int)blockIdx.x >= fb.f[t.f + 1].tbase) ++t.f;
    t.fa = &fb.f[t.f];
    const FrameDesc &fa = *t.fa;
    const int lt = (int)blockIdx.x - fa.tbase;
    const int tiles_x = (fa.Wq + kTX - 1) / kTX;
    t.qx0 = (lt % tiles_x) * kTX;
    t.qy0 = (lt / tiles_x) * kTY;
    t.nqx = min(kTX, fa.Wq - t.qx0);
    t.nqy = min(kTY, fa.Hq - t.qy0);
    const int rw = ((t.nqx - 1) * s + p) * C;   // bytes per region row
    const int rh = (t.nqy - 1) * s + p;
    t.ldw = ext_ldw(p, C, s);                   // LDS row pitch (fixed, whole words)
    const uint8_t *src = fa.frame + (int64_t)(t.qy0 * s) * fa.pitch + (int64_t)(t.qx0 * s) * C;
    // whole words where the frame rows allow it (the region's first byte and
    // the pitch word-aligned), then each row's last rw % 4 bytes; nothing is
    // read beyond a region row
    const bool wa = ((fa.pitch | reinterpret_cast<uintptr_t>(src)) & 3) == 0;
    const int nw = wa ? rw >> 2 : 0, tail = rw - 4 * nw;
    for (int e = threadIdx.x; e < nw * rh; e += kTX * kTY) {
        const int r = e / nw, c = e - r * nw;
        reinterpret_cast<uint32_t *>(s_tile + r * t.ldw)[c] =
            reinterpret_cast<const uint32_t *>(src + (int64_t)r * fa.pitch)[c];
    }
    for (int e = threadIdx.x; e < tail * rh; e += kTX * kTY) {
        const int r = e / tail, c = 4 * nw + (e - r * tail);
        s_tile[r * t.ldw + c] = src[(int64_t)r * fa.pitch + c];
    }
    __syncthreads();
    return t;
}

template <int DP>
__global__ __launch_bounds__(kTX *kTY) void k_extract(DevIndex ix, FrameBatch fb, Work w) {
    extern __shared__ uint8_t s_tile[];
    if (blockIdx.x == 0 && threadIdx.x < 4) w.counters[threadIdx.x] = 0u;   // ring/dense list counts
    const int p = ix.p, C = ix.C, s = ix.s, D = ix.D;
    const ExtTile t = load_tile(ix, fb, s_tile);
    const FrameDesc &fa = *t.fa;
    const int f = t.f, qx0 = t.qx0, qy0 = t.qy0, ldw = t.ldw;

    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    if (tx >= t.nqx || ty >= t.nqy) return;
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

// Window rows of P*C bytes, a whole number of words: row dy of the window
// starts at LDS byte b (its own alignment per row); the aligned words b/4 ..
// b/4 + PC/4 hold it, and v_alignbyte by b % 4 takes each output word from
// two of them.  The LDS allocation has a spare word for the last row's extra
// word, whose bytes beyond the row are shifted out.
template <int DP, int P, int C>
__global__ __launch_bounds__(kTX *kTY) void k_extract_rows(DevIndex ix, FrameBatch fb, Work w) {
    extern __shared__ __attribute__((aligned(16))) uint8_t s_tile[];
    if (blockIdx.x == 0 && threadIdx.x < 4) w.counters[threadIdx.x] = 0u;   // ring/dense list counts
    constexpr int PC = P * C, NW = PC / 4, D = P * PC;
    static_assert(PC % 4 == 0 && D <= DP, "whole-word window rows");
    const int s = ix.s;
    // 64-byte patches: each row of the tile is staged here and leaves as whole
    // contiguous kilobytes (four 16-byte stores per lane, lanes adjacent)
    constexpr bool kStage = DP == 64;
    __shared__ __attribute__((aligned(16))) uint4 s_out[kStage ? kTY * kTX * (DP / 16) : 1];
    const ExtTile t = load_tile(ix, fb, s_tile);
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const bool valid = tx < t.nqx && ty < t.nqy;
    if (!kStage && !valid) return;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(s_tile);
    const int base = (ty * s) * t.ldw + (tx * s) * C;
    uint32_t wd[DP / 4];
    int sa2 = 0, sa = 0;
#pragma unroll
    for (int dy = 0; dy < P; ++dy) {
        // each row has its own alignment (the LDS row pitch is any byte count)
        const int b = base + dy * t.ldw, a0 = b >> 2;
        const uint32_t sh = (uint32_t)(b & 3);
        uint32_t x[NW + 1];
#pragma unroll
        for (int j = 0; j <= NW; ++j) x[j] = words[a0 + j];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const uint32_t word = __builtin_amdgcn_alignbyte(x[j + 1], x[j], sh) ^ 0x7F7F7F7Fu;
            wd[dy * NW + j] = word;
            sa2 = __builtin_amdgcn_sdot4((int)word, (int)word, sa2, false);
            sa = __builtin_amdgcn_sdot4((int)word, 0x01010101, sa, false);
        }
    }
#pragma unroll
    for (int i = D / 4; i < DP / 4; ++i) wd[i] = 0u;
    const FrameDesc &fa = *t.fa;
    const int64_t q0 = fa.qbase + (int64_t)(t.qy0 + ty) * fa.Wq + t.qx0;   // row's first query
    const int64_t q = q0 + tx;
    if constexpr (kStage) {
        constexpr int PW = DP / 16;               // 16-byte words per patch
        uint4 *row = s_out + ty * (kTX * PW);
#pragma unroll
        for (int i = 0; i < PW; ++i)
            row[tx * PW + i] = make_uint4(wd[4 * i], wd[4 * i + 1], wd[4 * i + 2], wd[4 * i + 3]);
        __syncthreads();
        if (ty < t.nqy) {
            uint4 *dst = reinterpret_cast<uint4 *>(w.patches + q0 * DP);
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const int g = i * kTX + tx;           // word g of the row: patch g / PW
                if (g / PW < t.nqx) dst[g] = row[g];
            }
        }
        if (!valid) return;
    } else {
        uint4 *dst = reinterpret_cast<uint4 *>(w.patches + q * DP);
#pragma unroll
        for (int i = 0; i < DP / 16; ++i)
            dst[i] = make_uint4(wd[4 * i], wd[4 * i + 1], wd[4 * i + 2], wd[4 * i + 3]);
    }
    w.qc[q] = sa2 + 2 * sa + D;
    w.fid[q] = (uint8_t)t.f;
}

template <int DP>
hipError_t launch_extract_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                            hipStream_t st) {
    const size_t lds = ext_lds_bytes(ix.p, ix.C, ix.s);
    const dim3 grid((unsigned)fb.ntiles), block(kTX * kTY);
    // whole-word window rows of the common shapes
    bool fast = false;
    if constexpr (DP == 64) {
        if ((fast = ix.p == 8 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 8, 1>), grid, block, lds,
                               st, ix, fb, w);
    } else if constexpr (DP == 192) {
        if ((fast = ix.p == 8 && ix.C == 3))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 8, 3>), grid, block, lds,
                               st, ix, fb, w);
    } else if constexpr (DP == 160) {
        if ((fast = ix.p == 12 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 12, 1>), grid, block, lds,
                               st, ix, fb, w);
    } else if constexpr (DP == 256) {
        if ((fast = ix.p == 16 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 16, 1>), grid, block, lds,
                               st, ix, fb, w);
    }
    if (!fast)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract<DP>), grid, block, lds, st, ix, fb, w);
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
