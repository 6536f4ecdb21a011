/*
 * riann.h -- C ABI of libriann: RIANN ANN fields on AMD Instinct MI355X (gfx950).
 *
 * Paper: Ben-Zrihem & Zelnik-Manor, "Approximate Nearest Neighbor Fields in
 * Video" (arXiv 1508.07953).  Problem statement (Sec. 1 and Fig. 1): a
 * reference set R of n patches is fixed for the whole video; for every frame,
 * every query patch q_{x,y,t} (Sec. 3.1) is matched to a reference patch,
 * giving a dense ANN field per frame.
 *
 * This library computes the field EXACTLY: idx(x,y) is the lowest reference
 * index among those at minimum squared L2 distance (SSD over raw uint8
 * values) from the query, and ssd(x,y) is that distance.  It gets there with
 * the paper's ring intersection (Sec. 3.2-3.4, Algorithm 1) in exact mode:
 * the radius R is the distance to the previous frame's match and is not
 * capped, and rings are drawn around K key points chosen from R.  Every
 * reference within R of the query lies in every ring (triangle inequality),
 * so the result never depends on the previous field; a poor or missing
 * previous match only costs time.  Queries whose smallest ring is large are
 * answered by an exact int8 matrix-core search instead.
 *
 * Conventions
 *   patches   p x p x C windows, flattened in (dy, dx, c) order; D = p*p*C,
 *             1 <= D <= 256.
 *   frames    H x W x C uint8, channels last, rows `pitch` bytes apart
 *             (pitch >= W*C), device memory.
 *   fields    Hq x Wq row-major, Hq = (H-p)/s + 1, Wq = (W-p)/s + 1; the query
 *             at field position (i, j) has its top-left corner at pixel
 *             (x, y) = (s*j, s*i).  Indices are 0-based int32.
 *   prev      previous frame's field (device, Hq x Wq int32).  An entry of -1
 *             or outside [0, n) means "no prior": that query's rings are the
 *             whole set.  prev may be NULL (every query without prior).
 *             prev must not alias out.
 *   streams   `hip_stream` is a hipStream_t (NULL = the default stream).
 *             match / full_search / batch calls only enqueue work on that
 *             stream and return; argument errors are reported synchronously;
 *             a device fault surfaces as RIANN_E_DEVICE from the next call
 *             that synchronises (riann_get_stats, riann_save, riann_destroy).
 *   graphs    match / full_search / batch calls can be captured into a HIP
 *             graph: the first call on a stream (or one with more queries
 *             than any before) allocates that stream's scratch, and later
 *             calls of up to that size allocate nothing, synchronise nothing
 *             and clear their counters with a kernel, not a memset.  Warm the
 *             capture stream with one call, then capture; a replay re-reads
 *             the captured frame/prev buffers and rewrites out/ssd.  The
 *             host-side frame counter of riann_get_stats counts the capture,
 *             not the replays.
 *   ownership the index owns device copies of the reference set and its
 *             tables; the caller owns frames and fields.
 *   threads   one index may be used from several host threads and streams at
 *             once; each stream gets its own scratch space.
 *   errors    no exceptions cross this ABI; every call returns a status and
 *             riann_last_error() gives a message for the calling thread.
 */
#ifndef RIANN_H
#define RIANN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct riann_index *riann_index_t;

typedef enum {
    RIANN_OK = 0,
    RIANN_E_INVALID = -1,      /* bad argument, shape, alias or state        */
    RIANN_E_NOMEM = -2,        /* device or host allocation failed           */
    RIANN_E_DEVICE = -3,       /* HIP runtime / kernel error                  */
    RIANN_E_UNSUPPORTED = -4,  /* valid request this build does not support  */
    RIANN_E_IO = -5            /* file error in save / load                   */
} riann_status_t;

typedef struct riann_params {
    int32_t patch;             /* p, patch side in pixels (Sec. 4 uses 8)     */
    int32_t channels;          /* C, 1 (gray) or 3 (RGB)                       */
    int32_t stride;            /* s, step between query windows (>= 1)        */
    int32_t n_keys;            /* K, number of key points (0 <= K <= 64)      */
    int64_t n_ref;             /* n, number of reference patches (>= 1)       */
    int64_t dense_threshold;   /* queries whose smallest ring holds more than
                                  this many candidates use the dense search;
                                  < 0 selects the library default             */
    uint32_t flags;            /* RIANN_FLAG_* bits, else 0                    */
    uint32_t reserved;         /* must be 0                                    */
} riann_params_t;

/* riann_params_t.flags: answer dense queries with the column-layout search
 * (queries as MFMA rows) instead of the default row layout (references as
 * MFMA rows).  Results are identical; this exists for measurement and as a
 * cross-check of the two kernels. */
#define RIANN_FLAG_COLUMN_DENSE 1u

/* riann_params_t.flags: evaluate the smallest ring m* of every ring-phase
 * query exactly.  By default a query whose ring-size lower bounds (per-key
 * bucket counts of the sorted distance lists, Sec. 3.3) already exceed the
 * dense threshold on every key goes to the dense search without its exact
 * m*: its smallest ring holds more than the threshold's candidates either
 * way, so routing and results are identical; only riann_stats_t.sum_mstar
 * then leaves such queries out (they are counted in bound_routed). */
#define RIANN_FLAG_EXACT_MSTAR 2u

/* riann_params_t.flags: scan rings by gathering each candidate's pivot row
 * (one K-word row per reference, reached through the sorted list's index)
 * instead of the default ring-ordered copy, in which entry j of key k's
 * sorted list carries its reference's whole pivot row (Sec. 3.3 tables laid
 * out so that scanning a ring is one contiguous read).  The default costs
 * K * n * 4 * KR more bytes of device memory (KR = 8, 16, 32, 48 or 64 words
 * for K <= 8, 16, 32, 48, 64: 16 MB at n = 16,384, K = 16; 2.4 GB at
 * n = 262,144, K = 48); results are identical. */
#define RIANN_FLAG_GATHER_SCAN 4u

/* One frame of a batch (riann_match_batch). */
typedef struct riann_frame_desc {
    const uint8_t *frame;      /* device, H x W x C, row pitch `pitch`         */
    int32_t H, W;
    int64_t pitch;
    const int32_t *prev;       /* device Hq x Wq, or NULL (no prior); ignored
                                  when mode == RIANN_MODE_FULL                 */
    int32_t *out;              /* device Hq x Wq                               */
    uint32_t *ssd;             /* device Hq x Wq (may be NULL)                 */
    int32_t mode;              /* RIANN_MODE_RING or RIANN_MODE_FULL           */
    int32_t reserved;
} riann_frame_desc_t;

#define RIANN_MODE_RING 0
#define RIANN_MODE_FULL 1

/* Counters accumulated by every match call since build/load or the last
 * riann_reset_stats.  Ring statistics follow the paper's observation that
 * more temporal change means larger rings and more work (Sec. 3.3, Fig. 4). */
typedef struct riann_stats {
    uint64_t frames;           /* frames processed                             */
    uint64_t queries;          /* query patches processed                      */
    uint64_t ring_queries;     /* queries answered by the ring scan            */
    uint64_t dense_queries;    /* queries answered by the dense search         */
    uint64_t no_prior;         /* queries whose prev entry was -1/out of range  */
    uint64_t sum_mstar;        /* sum over ring-phase queries (all queries of
                                  RING frames) of the smallest ring size m*,
                                  except those in bound_routed                 */
    uint64_t sum_survivors;    /* sum over ring-scanned queries of |S|, the
                                  number of references inside all K rings     */
    uint64_t sum_mstar_ring;   /* sum of m* over ring-scanned queries only     */
    uint64_t bound_routed;     /* ring-phase queries sent to the dense search
                                  by their ring-size lower bounds alone, m*
                                  not evaluated (0 with RIANN_FLAG_EXACT_MSTAR) */
    uint64_t dense_routed;     /* ring-phase queries routed to the dense search
                                  (dense_queries without the queries of
                                  full-search frames)                          */
    uint64_t bsearch_probes;   /* sorted-table reads of the ring phase's binary
                                  searches (Sec. 3.3: a ring costs two
                                  O(log n) searches): one per LDS sample probed,
                                  per line start probed in device memory and per
                                  64-byte line counted                         */
} riann_stats_t;

/*
 * riann_build -- pre-processing (Sec. 3.3 and Sec. 3.4 "Building a reference
 * model"): copy the reference set to the device and build, for each key
 * point k, the ascending list of distances SSD(r, k) over all references r
 * (with the matching reference indices; ties ordered by index), plus the
 * n x K table SSD(r, k).  The paper sorts the full n x n matrix; this library
 * keeps only K columns of it, so memory is O(K n) instead of O(n^2).
 *
 *   ref_host   host, n x D uint8, row-major, (dy, dx, c) patch order
 *   key_idx    host, K distinct indices in [0, n) (the key points)
 *   p          shapes and options (see riann_params_t)
 *   hip_stream stream used for the uploads (the call synchronises it)
 *   out        receives the new index; unchanged on error
 * Returns RIANN_E_INVALID for bad shapes or duplicate/out-of-range keys,
 * RIANN_E_NOMEM if device memory is short.
 */
riann_status_t riann_build(const uint8_t *ref_host, const int32_t *key_idx,
                           const riann_params_t *p, void *hip_stream,
                           riann_index_t *out);

/*
 * riann_match_frame -- the online search of Algorithm 1 for one frame, in
 * exact mode.  For every query patch q of `frame`:
 *   c   = SSD(q, R[prev])            radius^2 from the previous match
 *   b_k = SSD(q, key_k)              distance to each key point
 *   ring k = { r : |d(r,k) - d(q,k)| <= sqrt(c) }, closed, found by two
 *            binary searches in key k's sorted list (Sec. 3.3)
 *   S   = references in every ring, scanned from the smallest ring
 *   out = arg min over S of SSD(q, r) (lowest index on ties), ssd = the min.
 * Queries whose smallest ring is larger than the dense threshold are answered
 * by the exact dense search instead (same result).
 *
 *   frame_dev  device H x W x C uint8 with row pitch `pitch` bytes
 *   prev_dev   device Hq x Wq int32 or NULL; must not overlap out_dev
 *   out_dev    device Hq x Wq int32 (written)
 *   ssd_dev    device Hq x Wq uint32 (written) or NULL
 * Asynchronous on hip_stream.
 */
riann_status_t riann_match_frame(riann_index_t h, const uint8_t *frame_dev,
                                 int32_t H, int32_t W, int64_t pitch,
                                 const int32_t *prev_dev, int32_t *out_dev,
                                 uint32_t *ssd_dev, void *hip_stream);

/*
 * riann_match_frame_noalloc -- riann_match_frame for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same kernels and the
 * same result as riann_match_frame, but the per-frame scratch (query
 * patches, ring records, route lists and their counters) lives in one
 * static device array of 64 MiB per GPU, held from the library's load until
 * the process ends; this call allocates nothing.  The array holds the
 * scratch of frames with up to about 470,000 queries at D = 64 (a
 * 640 x 720 gray frame at stride 1) or 250,000 at D = 192 (640 x 360 RGB);
 * a larger frame returns RIANN_E_UNSUPPORTED with the bytes it needs.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (other streams, other threads, other indexes) race and must be ordered by
 * the caller.  The list counters a call uses are cleared by its own
 * extraction kernel (a call that needs no extraction uses none).
 * Kernel timing (riann_set_profiling) is not recorded for this call.
 */
riann_status_t riann_match_frame_noalloc(riann_index_t h, const uint8_t *frame_dev,
                                         int32_t H, int32_t W, int64_t pitch,
                                         const int32_t *prev_dev, int32_t *out_dev,
                                         uint32_t *ssd_dev, void *hip_stream);

/*
 * riann_full_search -- exact nearest neighbour of every query by exhaustive
 * search (the exact NN the paper uses for its analyses, Sec. 3.1), used for
 * the first frame (Algorithm 1 starts from a random field instead) and at
 * scene cuts.  Runs as an int8 matrix-core GEMM on 128-shifted patches with
 * int32 accumulation; all distances are exact integers.
 * Arguments as riann_match_frame without prev.  Asynchronous on hip_stream.
 */
riann_status_t riann_full_search(riann_index_t h, const uint8_t *frame_dev,
                                 int32_t H, int32_t W, int64_t pitch,
                                 int32_t *out_dev, uint32_t *ssd_dev,
                                 void *hip_stream);

/*
 * riann_match_batch -- several frames of possibly different sizes (one per
 * live stream) matched in one submission; each descriptor is processed as
 * riann_match_frame (mode RING) or riann_full_search (mode FULL).
 *   descs  host array of n descriptors (copied before return)
 * Asynchronous on hip_stream.  Output fields of different descriptors must
 * not overlap.
 */
riann_status_t riann_match_batch(riann_index_t h, const riann_frame_desc_t *descs,
                                 int32_t n, void *hip_stream);

/*
 * riann_match_knn -- exact k-nearest-neighbour field of one frame (the
 * Conclusion, Sec. 7, states that the method can return several closest
 * matches instead of one): for every query the k references with the
 * smallest (SSD, index), in ascending order.
 *   k       1..8; k <= n.  k = 1 is riann_match_frame / riann_full_search.
 *   prev    RING mode: device Hq x Wq x k, the previous frame's k-NN field, or
 *           NULL.  The ring radius is the largest SSD from the query to its k
 *           previous matches; those k references lie within it, so the k
 *           nearest do too and every one of them is inside every ring.  A
 *           query whose k entries are not k distinct indices in [0, n) has no
 *           radius (the exact result is still returned).  Ignored in FULL mode.
 *   out     device Hq x Wq x k int32;  ssd  device Hq x Wq x k uint32 or NULL
 *   mode    RIANN_MODE_RING or RIANN_MODE_FULL (exhaustive)
 * For k > 1 the dense search keeps 32-bit keys over the whole reference set.
 * The default row layout takes the class-ordered set (each parity class of
 * Rc padded to whole 32-row tiles, the whole to 512 rows) up to 2^b tiles,
 * b = 32 - ceil(log2(Dp * 81409 / 2 + 2)) with Dp = D rounded up to 32: about
 * 65,472 references for Dp = 32, 32,704 for Dp <= 96, 16,320 for Dp <= 192
 * and 8,128 for Dp <= 256.  With RIANN_FLAG_COLUMN_DENSE (or beyond those
 * sizes) the column layout takes n <= 32 * 2^jb (rounded up to 512),
 * jb = 32 - ceil(log2(81409 * D + 2)): 32768 for D <= 32, 16384 for D <= 64,
 * 8192 for D <= 192, 4096 for D <= 256.  Larger sets return
 * RIANN_E_UNSUPPORTED.
 * Asynchronous on hip_stream; prev must not overlap out or ssd.
 */
riann_status_t riann_match_knn(riann_index_t h, const uint8_t *frame, int32_t H, int32_t W,
                               int64_t pitch, int32_t k, const int32_t *prev, int32_t *out,
                               uint32_t *ssd, int32_t mode, void *hip_stream);

/*
 * riann_footprint -- device bytes an index with parameters p needs, plus the
 * per-stream scratch for frames of H x W (H = W = 0: index only).  An upper
 * bound: the dense search's class-ordered copy of the references is counted
 * with the most padding any reference set of n can need.
 */
riann_status_t riann_footprint(const riann_params_t *p, int32_t H, int32_t W,
                               int64_t *bytes);

/*
 * The paper's own approximate search (Algorithm 1), for comparison with the
 * exact search.  Patches are raw uint8 (no unit normalisation), distances are
 * integer SSDs, and alpha = 1/4, so the fat ring d -/+ alpha*d around a
 * reference r at query distance d is 9*SSD(q,r) <= 16*SSD(r,r_j) <=
 * 25*SSD(q,r).  Per query: r_i = prev entry (outside [0, n), or prev NULL: a
 * random reference drawn from the generator below); S = the ring of r_i,
 * preceded by r_i itself when SSD(q, r_i) > 0; while |S| >= L and some member
 * has not yet been an anchor: draw u = g(seed, t, q, iteration) mod (number
 * of members not yet drawn), take the u-th such member in S order as anchor
 * r_k and intersect S with r_k's ring -- unless that leaves nothing, which
 * stops the loop with S kept; the answer is the (SSD, index) minimum over S.
 * g is the SplitMix64 output function (Steele, Lea and Flood 2014) chained
 * over the counters: g = sm(sm(sm(sm(seed) ^ t) ^ q) ^ it), q = the query's
 * row-major field index (it = 2^32 - 1 draws the random initial match).
 *
 * riann_build_paper_tables -- pre-processing (Sec. 3.3): the n x n SSD
 *   matrix of the references and every row sorted by (value, index), built on
 *   the host and kept on the device (12 n^2 bytes; n <= 32768, else
 *   RIANN_E_UNSUPPORTED).  Synchronous.  Needed once per index.
 * riann_match_paper -- one frame; out/ssd Hq x Wq as for riann_match_frame;
 *   iters (device Hq x Wq int32, or NULL) receives the anchors drawn per
 *   query; L >= 1 (the paper uses 20); t is the frame number.  Asynchronous.
 */
riann_status_t riann_build_paper_tables(riann_index_t h, void *hip_stream);
riann_status_t riann_match_paper(riann_index_t h, const uint8_t *frame, int32_t H, int32_t W,
                                 int64_t pitch, const int32_t *prev, int32_t *out, uint32_t *ssd,
                                 int32_t *iters, int32_t L, uint64_t seed, uint64_t t,
                                 void *hip_stream);

/*
 * riann_stack_frames -- spatio-temporal patches (the 3D extension of Sec. 1).
 * Interleaves T frames into one H x W x (T*C) frame whose channel t*C + c is
 * channel c of frames[t], so that a p x p patch of the result is the
 * p x p x T space-time patch in (dy, dx, t, c) order.  An index built with
 * channels = T*C on such patches then matches space-time patches with every
 * other call unchanged.
 *   frames  host array of T device pointers (oldest first), each H x W x C
 *           uint8 with row pitch `pitch` bytes; 1 <= T <= 16
 *   out     device, H x W x (T*C) uint8, rows contiguous (pitch W*T*C); must
 *           not overlap any input frame
 * Asynchronous on hip_stream.  No index is needed.
 */
riann_status_t riann_stack_frames(const uint8_t *const *frames, int32_t T, int32_t H, int32_t W,
                                  int32_t C, int64_t pitch, uint8_t *out, void *hip_stream);

/*
 * riann_reconstruct -- rebuild a frame from its ANN field (Sec. 4: replace
 * every query patch by its match and average overlapping patches) or apply a
 * transformation through the field (Sec. 5: replace every query patch by the
 * transformed version of its match, T(R) computed by the caller).
 *   field         device, Hq x Wq int32 field of an H x W frame (Hq, Wq from
 *                 the index's patch and stride, as for riann_match_frame);
 *                 entries outside [0, n) contribute no patch
 *   app           device, n x (p*p*app_channels) uint8 appearance patches in
 *                 (dy, dx, c) order, or NULL for the index's own references
 *   app_channels  1..4; must equal the index's channels when app is NULL
 *   out           device, H x W x app_channels float32:
 *                 out = (sum of the covering patches' values) / (their count),
 *                 one float division; 0 where no patch covers the pixel (right
 *                 and bottom borders when the stride does not reach them)
 *   gt, gt_pitch  device H x W x app_channels uint8 with a row pitch in bytes,
 *                 or NULL; the reference frame for the error
 *   err           device, 4 doubles, or NULL (requires gt): {E, sum (gt-out)^2,
 *                 sum gt^2, number of values}, over covered pixels, with the
 *                 normalised error E = sqrt(err[1] / err[2]) (0 if err[2] = 0),
 *                 reduced in a fixed order (deterministic)
 * Asynchronous on hip_stream.  out must not overlap the inputs.  The first
 * call with err on a stream (or a larger frame) allocates a small scratch.
 */
riann_status_t riann_reconstruct(riann_index_t h, const int32_t *field, int32_t H, int32_t W,
                                 const uint8_t *app, int32_t app_channels, float *out,
                                 const uint8_t *gt, int64_t gt_pitch, double *err,
                                 void *hip_stream);

/* riann_get_stats -- synchronises the device and copies the counters. */
riann_status_t riann_get_stats(riann_index_t h, riann_stats_t *s);
riann_status_t riann_reset_stats(riann_index_t h);

/* riann_get_params -- the parameters the index was built with, with the
 * dense threshold resolved to the value in use. */
riann_status_t riann_get_params(riann_index_t h, riann_params_t *p);

/*
 * riann_set_dense_threshold -- change the routing threshold (queries whose
 * smallest ring holds more than `threshold` candidates use the dense search)
 * for launches issued after the call; threshold >= 0.  Routing never changes
 * a result, only the time it takes (the autotuner picks this value).  At 0
 * no query can be ring-scanned (every ring holds the nearest neighbour, so
 * m* >= 1): the ring phase is not run and every query with a previous match
 * is counted as bound_routed.
 */
riann_status_t riann_set_dense_threshold(riann_index_t h, int64_t threshold);

/*
 * riann_set_dense_shape -- block shape of the row-layout dense search (the
 * default; not RIANN_FLAG_COLUMN_DENSE) for launches issued after the call:
 * `waves` wavefronts per block and `cols` 32-query column blocks per
 * wavefront, i.e. 32 * cols queries per wavefront and 32 * cols * waves per
 * block.  waves = cols = 0 restores the patch width's default.  Only the
 * shapes riann_get_dense_shapes lists for the index's patch width are built;
 * any other returns RIANN_E_UNSUPPORTED.  The shape never changes a result,
 * only the time it takes (the autotuner picks it).
 */
riann_status_t riann_set_dense_shape(riann_index_t h, int32_t waves, int32_t cols);

/*
 * riann_get_dense_shapes -- the shapes built for the index's patch width,
 * the default first: writes up to `max` (waves, cols) pairs to the host
 * arrays waves[] and cols[] (either may be NULL), their number to *count and
 * the index of the shape in use to *current (either may be NULL).
 */
riann_status_t riann_get_dense_shapes(riann_index_t h, int32_t *waves, int32_t *cols,
                                      int32_t max, int32_t *count, int32_t *current);

/*
 * riann_save / riann_load -- write / read the index (reference set, keys and
 * tables) to / from a file, so the pre-processing is paid once
 * (Sec. 4: a single pre-processed global model serves many videos).
 * riann_save synchronises the device.  riann_load uploads on hip_stream and
 * synchronises it.  Format: little-endian binary, versioned header.
 */
riann_status_t riann_save(riann_index_t h, const char *path);
riann_status_t riann_load(const char *path, void *hip_stream, riann_index_t *out);

/* riann_destroy -- synchronises the device and frees the index. */
riann_status_t riann_destroy(riann_index_t h);

/*
 * Kernel timing (diagnostics).  riann_set_profiling(h, level): 0 turns it off;
 * RIANN_PROFILE_ALL brackets every kernel the index launches by two HIP
 * events recorded on the launch stream; RIANN_PROFILE_DENSE brackets only the
 * dense search (RIANN_K_DENSE, RIANN_K_FULL), which keeps the markers out of
 * the rest of a frame.  Turning it on synchronises the device and resets the
 * totals; other levels return RIANN_E_INVALID.  riann_get_profile synchronises, converts the pending event
 * pairs into milliseconds and returns the totals per kernel since profiling
 * was turned on.  Events are reused across calls.
 * Kernels: RIANN_K_RING (ring phase; with the default ring-ordered pivot
 * rows and the row-layout dense search it also runs the ring scan of its
 * ring-routed queries), RIANN_K_SCAN (ring scan and verification as a launch
 * of its own: RIANN_FLAG_GATHER_SCAN, RIANN_FLAG_COLUMN_DENSE or k-NN
 * fields), RIANN_K_DENSE (dense search of routed queries), RIANN_K_FULL
 * (dense search of whole frames), RIANN_K_EXTRACT (patch extraction, run
 * first for every frame; in a ring launch it also routes queries).  A
 * one-frame launch whose every query goes dense -- a full search, or a ring
 * frame at routing threshold 0 -- with 8x8 one-channel patches runs no
 * extraction: its dense search cuts the patches from the frame itself (and
 * counts the routing), so only RIANN_K_FULL or RIANN_K_DENSE records it.
 */
#define RIANN_K_RING 0
#define RIANN_K_SCAN 1
#define RIANN_K_DENSE 2
#define RIANN_K_FULL 3
#define RIANN_K_EXTRACT 4
#define RIANN_K_COUNT 5
#define RIANN_PROFILE_ALL 1
#define RIANN_PROFILE_DENSE 2
typedef struct riann_profile {
    uint64_t launches[RIANN_K_COUNT];
    double ms[RIANN_K_COUNT];
} riann_profile_t;
riann_status_t riann_set_profiling(riann_index_t h, int enable);
riann_status_t riann_get_profile(riann_index_t h, riann_profile_t *out);

/* Message for the last non-OK status returned on the calling thread. */
const char *riann_last_error(void);

/* ABI version, (major << 16) | minor. */
uint32_t riann_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RIANN_H */
