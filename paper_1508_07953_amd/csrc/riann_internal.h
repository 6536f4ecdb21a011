// riann_internal.h -- device-side layout of an index and the launch
// functions shared by the host API (api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace riann {

// Patch byte encodings used by every kernel (all exact integer arithmetic):
//   reference side  v = r - 128           (stored byte: r ^ 0x80, as int8)
//   query side      a = 127 - q           (byte: q ^ 0x7F, as int8)
// so q - r = -(a + v + 1) and, summing over the D real bytes,
//   SSD(q, r) = Qc(q) + Rc(r) + 2 <a, v>
//   Qc = sum (a + 1)^2,   Rc = sum v (v + 2).
// Padding bytes (k >= D) are 0 on both sides and add nothing.
constexpr int kTile = 32;        // references per dense tile (MFMA columns)
constexpr int kRefAlign = 512;   // n is padded to whole 16-tile dense stages
constexpr int kRowAlign = 256;   // row-layout references: whole 8-tile stages
// Row-layout dense search: a query's running minimum over a segment of
// 2^row_tile_bits(Dp) tiles is the key (Y << bits) | tile; every real Y is
// below row_pad_y(Dp) = 2^(32 - bits) - 1 (Y <= Dp * 81409 / 2), the value
// padding rows get.  A launch splits the reference range over at most
// kRowMaxParts blocks per query chunk.
__host__ __device__ constexpr int row_y_bits(int Dp) {
    int b = 1;
    while (((int64_t)1 << b) < (int64_t)Dp * 81409 / 2 + 2) ++b;
    return b;
}
__host__ __device__ constexpr int row_tile_bits(int Dp) { return 32 - row_y_bits(Dp); }
__host__ __device__ constexpr int32_t row_pad_y(int Dp) {
    return (int32_t)(((int64_t)1 << row_y_bits(Dp)) - 1);
}
constexpr int kRowMaxParts = 4;

// Ring-size lower bounds (k_ring): buckets per key and the padded row length
// (vmin, shift, cdf[0..B]); a table of at most ~8.5 KB for K <= 64.
__host__ __device__ constexpr int lb_buckets(int K) { return K <= 16 ? 128 : (K <= 32 ? 64 : 32); }
__host__ __device__ constexpr int lb_stride(int K) { return (lb_buckets(K) + 3 + 3) / 4 * 4; }
constexpr int kMaxKeys = 64;
// Routing rows (DevIndex::Rt): buckets per key, row stride in words.
constexpr int kRouteBuckets = 128;
constexpr int kRouteStride = kRouteBuckets + 4;
constexpr int kMaxPatch = 16;    // p <= 16 (D = p*p*C <= 256)

// Dense-search key of a (query, reference) pair, unsigned 32-bit:
//   X   = SSD - Qc + bias = Rc + 2<a, v> + bias,  bias = D * 16384 >= max Qc
//   key = (X << jb) | j,   j = the reference's tile number inside a segment
// X < 2^(32 - jb) - 1 for every real reference (jb chosen per D), so the
// unsigned minimum of the keys is the lexicographic (SSD, index) minimum.
// Rk[r] = (Rc[r] + bias) << jb; padding rows get 2^32 - 2^jb, above every
// real key.  In the kernel key = (Rk[r] | j) + (acc << (jb + 1)).

struct DevIndex {
    const int8_t *Rv;     // n_pad x Dp, reference rows (v bytes), 16-B aligned rows
    const int32_t *Rc;    // n_pad, Rc per row (0 for padding rows)
    const int8_t *Rf;     // n_pad x Dp, the same bytes in MFMA fragment order:
                          // tile t, k-block kb, lane l -> 16 bytes of row
                          // 32t + (l & 31), columns 32kb + 16(l >> 5) .. +16,
                          // at byte offset ((t * Dp/32 + kb) * 64 + l) * 16
    const uint32_t *Rk;   // n_pad dense key bases (see above)
    // Row-layout dense search (references as MFMA rows, queries as columns),
    // over its own reference order: first every reference with even Rc, then
    // every one with odd Rc, index order within each class, each class padded
    // to whole tiles and the whole to kRowAlign (n_rows rows).  With
    // p = Rc & 1 constant per tile, the lexicographic (Y, tile) minimum lies
    // in the tile that holds the (SSD, index) minimum.
    //   Rfr  n_rows x Dp, those rows in MFMA fragment order (as Rf)
    //   Hf   n_rows, per tile t 32 entries ordered [g][r] = row 32t +
    //        8(r/4) + 4g + r%4, the row accumulator register r of lane group g
    //        holds: Hf = (Rc + bias - p) / 2, so that Y = Hf + <a, v> and
    //        SSD - Qc + bias = 2Y + p (exact); padding rows get
    //        row_pad_y(Dp), above every real Y
    //   Rci  n_rows, {Rc, reference index} per row in tile order ({0, -1}
    //        for padding rows)
    const int8_t *Rfr;
    const int32_t *Hf;
    const int2 *Rci;
    int64_t n_rows;
    const uint32_t *T;    // K x n16, SSD(key_k, r) ascending; each key's list is
                          // padded to whole 16-entry (64-byte) lines with
                          // 0xFFFFFFFF, above every ring bound
    const int32_t *P;     // K x n, reference index of each T entry
    const uint32_t *Piv;  // n x Kp, SSD(r, key_k); rows padded to Kp = 4*ceil(K/4)
                          // with zeros (padding keys get the bounds [0, 2^32-1])
    const uint32_t *PivR; // K x n16 x KR, ring-ordered pivot rows: PivR[k][j] =
                          // Piv[P[k][j]] widened to KR words with zeros
                          // (entries j >= n are zero rows); nullptr with
                          // RIANN_FLAG_GATHER_SCAN (the scan then gathers Piv)
    int32_t KR;           // PivR row length in words: 8, 16, 32, 48 or 64
    const uint32_t *Ts;   // K x ns binary-search samples Ts[k][i] = T[k][i * 16 * s0l],
                          // copied to LDS by the ring phase
    const uint32_t *Lb;   // K x lbS ring-size lower-bound rows {vmin, shift,
                          // cdf[0..lbB]}: cdf[j] = #{T[k] < vmin + j 2^shift};
                          // copied to LDS after the samples (ns rounded to 4)
    const uint32_t *Rt;   // K x rtS routing rows in square-root space: {origin o
                          // (fp32 bits), scale 2^-e (fp32 bits), F[0..kRouteBuckets]}
                          // with F[j] = #{T[k] entries a : sqrt(a) < o + j 2^e}
    int32_t rtS;          // Rt row stride in words
    const int32_t *keys;  // K key indices
    int64_t n, n_pad;
    int32_t D, Dp, K, p, C, s;
    int32_t jb;           // index bits of a dense key
    int32_t bias;         // D * 16384
    int32_t n16;          // per-key stride of T (n rounded up to 16)
    int32_t ns;           // samples per key
    int32_t s0l;          // sample stride in 16-entry lines
    int32_t Kp;           // Piv row stride
    int32_t lbB, lbS;     // lower-bound buckets per key, row stride in words
    int32_t exact_mstar;  // 1: every ring-phase query's smallest ring is evaluated
    int32_t row_waves;    // block shape of the row-layout dense search: wavefronts
    int32_t row_cols;     // per block, 32-query column blocks per wavefront (0, 0:
                          // the patch width's default); read on the host only
};

// One frame of a launch.  A launch takes up to kMaxBatch frames of any sizes;
// their queries are numbered globally, frame f owning [qbase, qbase + Hq*Wq).
constexpr int kMaxBatch = 40;
constexpr int kModeRing = 0, kModeFull = 1;

struct FrameDesc {
    const uint8_t *frame;    // H x W x C bytes, rows `pitch` apart
    const int32_t *prev;     // Hq x Wq previous field or nullptr (ring mode)
    int32_t *out;            // Hq x Wq
    uint32_t *ssd;           // Hq x Wq or nullptr
    int64_t pitch;
    int64_t qbase;           // first global query id
    int32_t H, W, Hq, Wq;
    int32_t mode;            // kModeRing / kModeFull
    int32_t tbase;           // first extraction tile of this frame
};

// Passed by value (kernel arguments), so a launch needs no descriptor copy
// and can be captured in a graph as is.
constexpr int32_t kDenseMasked = 1, kDenseInOrder = 2;

struct FrameBatch {
    int32_t n;               // frames
    int32_t ntiles;          // extraction tiles over all frames
    int64_t Q;               // queries over all frames
    int32_t all_full;        // every frame in full-search mode
    int32_t knn;             // neighbours per query (1: prev/out/ssd are Hq x Wq;
                             // k > 1: Hq x Wq x k, each row ascending)
    int32_t dense_masked;    // kDenseMasked: the dense search takes every query in
                             // order and skips those the ring scan answers (route
                             // code kRouteScan) instead of reading the dense list;
                             // kDenseInOrder: every query in order, none was
                             // ring-scanned; 0: the dense list
    int32_t fused = 0;       // 1: one frame, every query dense, no extraction
                             // launch: the dense search reads its patches from
                             // the frame itself (dense_fused_supported shapes)
    unsigned long long *stats = nullptr;  // routing counts of a fused ring frame
    FrameDesc f[kMaxBatch];
};

// extraction tile: 64 x 4 query positions
constexpr int kExtTX = 64, kExtTY = 4;

// per-stream scratch of one launch
struct Work {
    uint8_t *patches;    // Q x Dp encoded query patches (a = q ^ 0x7F, zero padded)
    int32_t *qc;         // Q, Qc of each query
    uint8_t *fid;        // Q, frame of each query within its launch
    uint8_t *route;      // Q, route code from the extraction kernel (kRoute*),
                         // written in launches with a ring phase
    uint4 *rec;          // Q ring records {c, kstar, st, en}, by query; after the
                         // ring scan, row-layout dense with a split reference
                         // range: part 0's result, by dense-list position
    uint4 *rec2;         // 3 x capacity, row-layout dense: parts 1..3 of a split
                         // reference range, likewise
    uint32_t *ring_list; // Q
    uint32_t *dense_list;// Q
    uint32_t *counters;  // [0] ring count, [1] dense count
    int64_t capacity;    // Q capacity
};

// Route codes the extraction kernel gives each query of a launch with a ring
// phase: kRouteRing leaves the query to the ring kernel; the others go to
// the dense search without it -- full-search frames, queries without a
// valid previous match, and queries whose every ring holds more than the
// routing threshold's candidates by the per-key bucket-count lower bounds.
// The ring kernel then marks the queries the ring scan answers kRouteScan.
enum : uint8_t { kRouteRing = 0, kRouteFull = 1, kRouteNoPrior = 2, kRouteBound = 3,
                 kRouteScan = 4 };

// device stats block (uint64 counters, same order as riann_stats_t after `frames`)
enum StatSlot {
    ST_QUERIES = 0, ST_RING, ST_DENSE, ST_NOPRIOR, ST_MSTAR, ST_SURV, ST_MSTAR_RING,
    ST_BOUND, ST_PROBES, ST_COUNT
};
// Each counter is kept as kStatReplicas partial sums, each on a cache line of
// its own: a block adds into the replica of its block index, so the atomics of
// a launch's thousands of blocks spread over many addresses instead of
// queuing on one; the host sums the replicas.
constexpr int kStatReplicas = 64;
constexpr int kStatStride = 16;              // uint64 words: 128 bytes apart
constexpr int kStatWords = ST_COUNT * kStatReplicas * kStatStride;
__device__ __forceinline__ void stat_add(unsigned long long *stats, int slot,
                                         unsigned long long v) {
    atomicAdd(stats + ((size_t)slot * kStatReplicas + blockIdx.x % kStatReplicas) * kStatStride,
              v);
}

// The hardware deals a launch's blocks to the chip's 8 XCDs (each with its
// own L2) in turn: block b runs on XCD b mod 8.  xcd_band(b, nb) maps block b
// of nb to the work item b / 8 of the (b mod 8)-th eighth of [0, nb) (a
// bijection), so each XCD works through one contiguous band of the items and
// its L2 holds what neighbouring items share.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_band(uint32_t b, uint32_t nb) {
    const uint32_t x = b % kXcds, per = nb / kXcds, rem = nb % kXcds;
    return x * per + min(x, rem) + b / kXcds;
}

// Extraction of every query patch; in launches with a ring phase also the
// route code of each query against `threshold` (the ring kernel's; < 0: no
// routing), and with fb.dense_masked the counts of what it routed (stats).
hipError_t launch_extract(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                          int64_t threshold, unsigned long long *stats, hipStream_t st);
hipError_t launch_ring(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                       unsigned long long *stats, int64_t threshold, hipStream_t st);
hipError_t launch_scan(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                       unsigned long long *stats, hipStream_t st);
// Ring-ordered pivot rows (k_ring.hip): the row length for K keys, and the
// device build of ix.PivR from ix.P and ix.Piv.
int pivr_words(int K);
// With the dense search reading route codes, one k-NN neighbour and the
// ring-ordered pivot rows, the ring kernel scans its own ring queries and no
// separate ring-scan launch follows.
bool ring_scans_inline(const DevIndex &ix, const FrameBatch &fb);
hipError_t launch_build_pivr(const DevIndex &ix, uint32_t *PivR, hipStream_t st);
// all_full batches: every query (no list); otherwise the dense list and its
// device-side count.  Reads the query patches written by launch_extract.
hipError_t launch_dense(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                        hipStream_t st);
// Row-layout dense search (ix.n_rows > 0): the row kernel, which checks its
// own candidates unless the reference range is split over several blocks,
// when a resolve kernel merges the parts first.
bool dense_rows_supported(const DevIndex &ix);
// Patch shapes whose row-layout dense search can assemble its query patches
// from the frame itself (8 x 8 gray): a one-frame full search, or a ring frame
// at routing threshold 0, then runs without the extraction launch.
bool dense_fused_supported(const DevIndex &ix);
hipError_t launch_dense_rows(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             hipStream_t st);
// The block shapes built for patch width Dp as (waves, cols) pairs, the
// default first; returns their number and writes at most `max` of them.
int dense_rows_shapes(int Dp, int *waves, int *cols, int max);
// The row kernel at the non-default shape ix.row_waves x ix.row_cols.
hipError_t launch_dense_rows_shape(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                   hipStream_t st);
// T planar frames (each H x W x C, common row pitch) -> one H x W x (T*C)
// frame whose channel t*C + c is channel c of frame t (k_extract.hip).
constexpr int kMaxStack = 16;
struct StackArgs {
    const uint8_t *f[kMaxStack];
    int T, H, W, C;
    int64_t pitch;
    uint8_t *out;
};
hipError_t launch_stack(const StackArgs &sa, hipStream_t st);

// Frame reconstruction (k_recon.hip): out = average of the appearance patches
// field[i][j] over the patches covering each pixel; app == nullptr uses the
// index's references (Ca == C).  With gt and partials set, one fp64 partial
// {sum (gt - out)^2, sum gt^2, values} per block is written and reduced into
// err[0..3] = {E, sum (gt - out)^2, sum gt^2, values}.
struct ReconArgs {
    const int32_t *field;   // Hq x Wq
    int Hq, Wq, H, W, Ca;
    const uint8_t *app;     // n x (p*p*Ca) or nullptr
    float *out;             // H x W x Ca
    const uint8_t *gt;      // H x W x Ca with row pitch gt_pitch, or nullptr
    int64_t gt_pitch;
    double *partials;       // 3 per block, or nullptr (no error)
};
int64_t recon_blocks(int H, int W);
hipError_t launch_recon(const DevIndex &ix, const ReconArgs &ra, double *err, hipStream_t st);

// k-NN fields (fb.knn = k in [2, kMaxKnn]): the ring kernel takes the radius
// from the k previous matches; these answer the ring list and the dense list
// with the k smallest (SSD, index) per query.  The dense search needs the
// unsegmented key (n_pad / 32 tiles <= 2^jb), see knn_dense_supported.
constexpr int kMaxKnn = 8;
hipError_t launch_scan_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                           unsigned long long *stats, hipStream_t st);
bool knn_dense_supported(const DevIndex &ix);
// Row-layout k-NN (k_dense_rows.hip): one key segment of tiles, see
// knn_rows_supported; same contract as launch_dense_knn.
bool knn_rows_supported(const DevIndex &ix);
hipError_t launch_dense_rows_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                                 hipStream_t st);
hipError_t launch_dense_knn(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                            hipStream_t st);

// The paper's approximate search (k_paper.hip, Algorithm 1, alpha = 1/4):
// Dm n x n SSD between references, T/P each row of Dm sorted by (value,
// index) -- values and indices; iters (optional) receives anchors per query.
constexpr int64_t kMaxPaperN = 32768;
struct PaperArgs {
    const uint32_t *Dm;
    const uint32_t *T;
    const int32_t *P;
    int32_t L;
    int32_t pad;
    uint64_t seed, t;
    int32_t *iters;
};
size_t paper_lds_bytes(int64_t n);
hipError_t launch_paper(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                        const PaperArgs &pa, hipStream_t st);

// Column-layout dense search of an explicit list with a device-side count.
hipError_t launch_dense_list(const DevIndex &ix, const FrameBatch &fb, const Work &w,
                             const uint32_t *list, const uint32_t *count, hipStream_t st);

}  // namespace riann
