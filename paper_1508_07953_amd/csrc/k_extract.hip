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
//
// In a launch with a ring phase each thread also routes its query while the
// patch is in its registers (Algorithm 1's first steps): a full-search frame
// or a missing previous match goes to the dense search; otherwise the radius
// c = SSD(q, R[prev]), every key distance b_k and each key's ring-size lower
// bound from its bucket counts (the ring kernel's own test) are computed, and
// a query whose every ring certainly holds more than the routing threshold's
// candidates goes to the dense search too.  That certainty comes from each
// key's routing row: counts of its sorted list over buckets of sqrt(a), so a
// ring -- sqrt(a) within sqrt(c) of sqrt(b) -- is bounded from inside by
// whole buckets after two square roots.  The ring kernel then works only
// on the queries left to it.
#include "riann_internal.h"
#include "ring_math.h"

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

// Routing tables staged in LDS after the frame region (at a 16-byte
// boundary): each key's routing row (kRouteStride words), the key rows
// (DP / 4 words each) and the keys' Rc.  Staged when the launch routes on
// bounds.
__host__ __device__ __forceinline__ size_t route_lds_offset(int p, int C, int s) {
    return (ext_lds_bytes(p, C, s) + 15) & ~(size_t)15;
}
__host__ __device__ __forceinline__ size_t route_lds_bytes(int K, int DP) {
    return (size_t)K * (kRouteStride + DP / 4 + 1) * 4;
}
__device__ __forceinline__ bool route_codes_on(const FrameBatch &fb, int64_t threshold) {
    return threshold >= 0 && !fb.all_full;
}
__device__ __forceinline__ bool route_tables_on(const DevIndex &ix, const FrameBatch &fb,
                                                int64_t threshold) {
    return route_codes_on(fb, threshold) && fb.knn == 1 && ix.K > 0 && !ix.exact_mstar;
}
// Below a threshold of 1 no ring can qualify: the exact nearest neighbour is
// within sqrt(c) of q, so by the triangle inequality it lies in every ring of
// radius sqrt(c) (the exact-mode rings of Sec. 3.2), m* >= 1 for a query with
// a previous match, and that bound alone sends it to the dense search; c and
// the key distances are not needed and the tables are not staged.
__device__ __forceinline__ bool route_bounds_on(const DevIndex &ix, const FrameBatch &fb,
                                                int64_t threshold) {
    return route_tables_on(ix, fb, threshold) && threshold >= 1;
}

template <int DP>
__device__ __forceinline__ void stage_route_tables(const DevIndex &ix, uint32_t *tab) {
    const int nlb = ix.K * kRouteStride;          // multiple of 4
    for (int i = threadIdx.x; i < nlb / 4; i += kTX * kTY)
        reinterpret_cast<uint4 *>(tab)[i] = reinterpret_cast<const uint4 *>(ix.Rt)[i];
    uint32_t *keys = tab + nlb;
    for (int i = threadIdx.x; i < ix.K * (DP / 16); i += kTX * kTY) {
        const int k = i / (DP / 16), part = i - k * (DP / 16);
        reinterpret_cast<uint4 *>(keys)[i] =
            reinterpret_cast<const uint4 *>(ix.Rv + (int64_t)ix.keys[k] * ix.Dp)[part];
    }
    for (int k = threadIdx.x; k < ix.K; k += kTX * kTY)
        keys[ix.K * (DP / 4) + k] = (uint32_t)ix.Rc[ix.keys[k]];
}

// The route of one query, in two steps so that its loads are in flight
// early.  route_begin (before the patch is assembled): the part decided
// without rings -- full-search frame, k-NN launch (the ring kernel takes the
// k-NN radius), no valid previous match, no bound routing in this launch --
// or kRouteNeedBounds, with the previous match's index, row and Rc loads
// issued.  route_finish: c = SSD(q, R[prev]) and every key's ring tested
// against the threshold with the key rows staged in LDS (v_dot4).
constexpr uint8_t kRouteNeedBounds = 0xFE;
template <int DP>
struct RoutePrefetch {
    uint8_t code = kRouteFull;
    uint4 row[DP / 16];
    int rc = 0;
};

template <int DP>
__device__ __forceinline__ void route_begin(const DevIndex &ix, const FrameBatch &fb,
                                            const FrameDesc &fa, int64_t ql, int64_t threshold,
                                            RoutePrefetch<DP> &rp) {
    if (fa.mode == kModeFull) { rp.code = kRouteFull; return; }
    if (fb.knn != 1) { rp.code = kRouteRing; return; }
    if (!fa.prev) { rp.code = kRouteNoPrior; return; }
    const int32_t pv = fa.prev[ql];
    if (pv < 0 || (int64_t)pv >= ix.n) { rp.code = kRouteNoPrior; return; }
    if (!route_tables_on(ix, fb, threshold)) { rp.code = kRouteRing; return; }
    if (threshold < 1) { rp.code = kRouteBound; return; }
    rp.code = kRouteNeedBounds;
    const uint4 *src = reinterpret_cast<const uint4 *>(ix.Rv + (int64_t)pv * ix.Dp);
#pragma unroll
    for (int i = 0; i < DP / 16; ++i) rp.row[i] = src[i];
    rp.rc = ix.Rc[pv];
}

template <int DP>
__device__ __forceinline__ uint8_t route_finish(const DevIndex &ix, const uint32_t (&a)[DP / 4],
                                                int Qc, int64_t threshold, const uint32_t *tab,
                                                const RoutePrefetch<DP> &rp) {
    if (rp.code != kRouteNeedBounds) return rp.code;
    int d = 0;
#pragma unroll
    for (int i = 0; i < DP / 16; ++i) {
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 0], (int)rp.row[i].x, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 1], (int)rp.row[i].y, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 2], (int)rp.row[i].z, d, false);
        d = __builtin_amdgcn_sdot4((int)a[4 * i + 3], (int)rp.row[i].w, d, false);
    }
    const uint32_t c = (uint32_t)(Qc + rp.rc + 2 * d);
    const float sc = sqrt_est((float)c);          // SSDs are below 2^24: exact as fp32
    const uint32_t *keys = tab + ix.K * kRouteStride, *krc = keys + ix.K * (DP / 4);
    for (int k = 0; k < ix.K; ++k) {
        const uint32_t b = (uint32_t)(Qc + (int)krc[k] +
                                      2 * dot_row<DP>(a, reinterpret_cast<const int8_t *>(
                                                             keys + k * (DP / 4))));
        // a ring that may hold no more than the threshold's candidates: the
        // ring kernel decides
        if ((int64_t)route_lower_bound(tab + k * kRouteStride, sqrt_est((float)b), sc) <= threshold)
            return kRouteRing;
    }
    return kRouteBound;
}

// With the dense search reading route codes (fb.dense_masked) this kernel
// also counts what it routed: per block, the queries, and those it sent to
// the dense search as full-search, no-prior (each with m* = n, the whole set
// as its ring) and bound-routed queries.  `code` is 0xFF for a thread
// without a query.  Every thread of the block calls it (one barrier).
__device__ __forceinline__ void count_routes(const DevIndex &ix, unsigned long long *stats,
                                             uint8_t code) {
    constexpr int kWv = kTX * kTY / 64;
    __shared__ unsigned long long s_rc[kWv][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long vq = __ballot(code != 0xFF), fu = __ballot(code == kRouteFull),
                             np = __ballot(code == kRouteNoPrior), bd = __ballot(code == kRouteBound);
    if (lane == 0) {
        s_rc[wv][0] = (unsigned long long)__popcll(vq);
        s_rc[wv][1] = (unsigned long long)__popcll(fu);
        s_rc[wv][2] = (unsigned long long)__popcll(np);
        s_rc[wv][3] = (unsigned long long)__popcll(bd);
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long v[4] = {0, 0, 0, 0};
        for (int i = 0; i < kWv; ++i)
            for (int j = 0; j < 4; ++j) v[j] += s_rc[i][j];
        const int slot[5] = {ST_QUERIES, ST_DENSE, ST_NOPRIOR, ST_MSTAR, ST_BOUND};
        const unsigned long long val[5] = {v[0], v[1] + v[2] + v[3], v[2],
                                           v[2] * (unsigned long long)ix.n, v[3]};
        if (val[threadIdx.x]) stat_add(stats, slot[threadIdx.x], val[threadIdx.x]);
    }
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
__global__ __launch_bounds__(kTX *kTY) void k_extract(DevIndex ix, FrameBatch fb, Work w,
                                                     int64_t threshold,
                                                     unsigned long long *__restrict__ stats) {
    extern __shared__ __attribute__((aligned(16))) uint8_t s_tile[];
    if (blockIdx.x == 0 && threadIdx.x < 4) w.counters[threadIdx.x] = 0u;   // ring/dense list counts
    const int p = ix.p, C = ix.C, s = ix.s, D = ix.D;
    uint32_t *tab = reinterpret_cast<uint32_t *>(s_tile + route_lds_offset(p, C, s));
    if (route_bounds_on(ix, fb, threshold)) stage_route_tables<DP>(ix, tab);
    const ExtTile t = load_tile(ix, fb, s_tile);
    const FrameDesc &fa = *t.fa;
    const int f = t.f, qx0 = t.qx0, qy0 = t.qy0, ldw = t.ldw;

    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const bool valid = tx < t.nqx && ty < t.nqy;
    const bool codes = route_codes_on(fb, threshold);
    const int64_t q = fa.qbase + (int64_t)(qy0 + ty) * fa.Wq + (qx0 + tx);
    RoutePrefetch<DP> rp;
    if (valid && codes) route_begin<DP>(ix, fb, fa, q - fa.qbase, threshold, rp);
    uint8_t code = 0xFF;
    if (valid) {
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
                if (dy >= p) dy = p - 1;         // k >= D: stay inside the window
            }
            wd[i] = word;
            sa2 = __builtin_amdgcn_sdot4((int)word, (int)word, sa2, false);
            sa = __builtin_amdgcn_sdot4((int)word, 0x01010101, sa, false);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(w.patches + q * DP);
#pragma unroll
        for (int i = 0; i < DP / 16; ++i)
            dst[i] = make_uint4(wd[4 * i], wd[4 * i + 1], wd[4 * i + 2], wd[4 * i + 3]);
        // padding bytes are a = 0 and add nothing to the sums
        const int Qc = sa2 + 2 * sa + D;
        w.qc[q] = Qc;
        w.fid[q] = (uint8_t)f;
        if (codes) {
            code = route_finish<DP>(ix, wd, Qc, threshold, tab, rp);
            w.route[q] = code;
        }
    }
    if (fb.dense_masked && codes) count_routes(ix, stats, code);
}

// Window rows of P*C bytes, a whole number of words: row dy of the window
// starts at LDS byte b (its own alignment per row); the aligned words b/4 ..
// b/4 + PC/4 hold it, and v_alignbyte by b % 4 takes each output word from
// two of them.  The LDS allocation has a spare word for the last row's extra
// word, whose bytes beyond the row are shifted out.
template <int DP, int P, int C>
__global__ __launch_bounds__(kTX *kTY) void k_extract_rows(DevIndex ix, FrameBatch fb, Work w,
                                                          int64_t threshold,
                                                          unsigned long long *__restrict__ stats) {
    extern __shared__ __attribute__((aligned(16))) uint8_t s_tile[];
    if (blockIdx.x == 0 && threadIdx.x < 4) w.counters[threadIdx.x] = 0u;   // ring/dense list counts
    uint32_t *tab = reinterpret_cast<uint32_t *>(s_tile + route_lds_offset(P, C, ix.s));
    if (route_bounds_on(ix, fb, threshold)) stage_route_tables<DP>(ix, tab);
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
    const FrameDesc &fa = *t.fa;
    const int64_t q0 = fa.qbase + (int64_t)(t.qy0 + ty) * fa.Wq + t.qx0;   // row's first query
    const int64_t q = q0 + tx;
    // the previous match's row and Rc are fetched while the patch is built
    const bool codes = route_codes_on(fb, threshold);
    RoutePrefetch<DP> rp;
    if (valid && codes) route_begin<DP>(ix, fb, fa, q - fa.qbase, threshold, rp);
    // every thread assembles a window (those without a query read inside the
    // tile's LDS region and write nothing): the staging and the route counts
    // below take the whole block
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
    } else if (valid) {
        uint4 *dst = reinterpret_cast<uint4 *>(w.patches + q * DP);
#pragma unroll
        for (int i = 0; i < DP / 16; ++i)
            dst[i] = make_uint4(wd[4 * i], wd[4 * i + 1], wd[4 * i + 2], wd[4 * i + 3]);
    }
    uint8_t code = 0xFF;
    if (valid) {
        const int Qc = sa2 + 2 * sa + D;
        w.qc[q] = Qc;
        w.fid[q] = (uint8_t)t.f;
        if (codes) {
            code = route_finish<DP>(ix, wd, Qc, threshold, tab, rp);
            w.route[q] = code;
        }
    }
    if (fb.dense_masked && codes) count_routes(ix, stats, code);
}

template <int DP>
hipError_t launch_extract_t(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                            int64_t threshold, unsigned long long *stats, hipStream_t st) {
    const bool tables = threshold >= 1 && !fb.all_full && fb.knn == 1 && ix.K > 0 &&
                        !ix.exact_mstar;
    const size_t lds = tables ? route_lds_offset(ix.p, ix.C, ix.s) + route_lds_bytes(ix.K, DP)
                              : ext_lds_bytes(ix.p, ix.C, ix.s);
    const dim3 grid((unsigned)fb.ntiles), block(kTX * kTY);
    // whole-word window rows of the common shapes
    bool fast = false;
    if constexpr (DP == 64) {
        if ((fast = ix.p == 8 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 8, 1>), grid, block, lds,
                               st, ix, fb, w, threshold, stats);
    } else if constexpr (DP == 192) {
        if ((fast = ix.p == 8 && ix.C == 3))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 8, 3>), grid, block, lds,
                               st, ix, fb, w, threshold, stats);
    } else if constexpr (DP == 160) {
        if ((fast = ix.p == 12 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 12, 1>), grid, block, lds,
                               st, ix, fb, w, threshold, stats);
    } else if constexpr (DP == 256) {
        if ((fast = ix.p == 16 && ix.C == 1))
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract_rows<DP, 16, 1>), grid, block, lds,
                               st, ix, fb, w, threshold, stats);
    }
    if (!fast)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_extract<DP>), grid, block, lds, st, ix, fb, w,
                           threshold, stats);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_extract(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          int64_t threshold, unsigned long long *stats, hipStream_t st) {
    switch (ix.Dp) {
    case 32: return launch_extract_t<32>(ix, fb, w, threshold, stats, st);
    case 64: return launch_extract_t<64>(ix, fb, w, threshold, stats, st);
    case 96: return launch_extract_t<96>(ix, fb, w, threshold, stats, st);
    case 128: return launch_extract_t<128>(ix, fb, w, threshold, stats, st);
    case 160: return launch_extract_t<160>(ix, fb, w, threshold, stats, st);
    case 192: return launch_extract_t<192>(ix, fb, w, threshold, stats, st);
    case 224: return launch_extract_t<224>(ix, fb, w, threshold, stats, st);
    case 256: return launch_extract_t<256>(ix, fb, w, threshold, stats, st);
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
