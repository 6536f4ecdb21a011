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
constexpr int32_t kBias = 1 << 22;                 // >= max Qc for D <= 256
constexpr int32_t kRcPad = (1 << 26) - 1 - kBias;  // Rc of padding rows: never wins
constexpr int kTile = 32;                           // references per dense tile
constexpr int kMaxKeys = 64;

struct DevIndex {
    const int8_t *Rv;     // n_pad x Dp, reference rows (v bytes), 16-B aligned rows
    const int32_t *Rc;    // n_pad, Rc per row (kRcPad for rows >= n)
    const uint32_t *T;    // K x n, SSD(key_k, r) ascending
    const int32_t *P;     // K x n, reference index of each T entry
    const uint32_t *Piv;  // n x K, SSD(r, key_k)
    const int32_t *keys;  // K key indices
    int64_t n, n_pad;
    int32_t D, Dp, K, p, C, s;
};

struct FrameArgs {
    const uint8_t *frame;
    int64_t pitch;
    int32_t H, W, Hq, Wq;
};

// per-stream scratch of one frame
struct Work {
    uint4 *rec;          // Q records {c, kstar, st, en}
    uint32_t *ring_list; // Q
    uint32_t *dense_list;// Q
    uint32_t *counters;  // [0] ring count, [1] dense count
    int64_t capacity;    // Q capacity
};

// device stats block (uint64 counters, same order as riann_stats_t after `frames`)
enum StatSlot {
    ST_QUERIES = 0, ST_RING, ST_DENSE, ST_NOPRIOR, ST_MSTAR, ST_SURV, ST_MSTAR_RING,
    ST_COUNT
};

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st);
hipError_t launch_ring(const DevIndex &ix, const FrameArgs &fa, const int32_t *prev,
                       const Work &w, unsigned long long *stats, int64_t threshold,
                       hipStream_t st);
hipError_t launch_scan(const DevIndex &ix, const FrameArgs &fa, const Work &w,
                       int32_t *out, uint32_t *ssd, unsigned long long *stats,
                       hipStream_t st);
// list == nullptr: all Q queries (count_static); otherwise list/count_dev
hipError_t launch_dense(const DevIndex &ix, const FrameArgs &fa, const uint32_t *list,
                        const uint32_t *count_dev, uint32_t count_static, int32_t *out,
                        uint32_t *ssd, hipStream_t st);

}  // namespace riann
