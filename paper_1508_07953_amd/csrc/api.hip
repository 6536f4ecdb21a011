// api.hip -- host side of libriann: argument checking, the pre-processing
// (sorted key-distance tables, Sec. 3.3), per-stream scratch and the launch
// sequence of each entry point declared in include/riann.h.
#include "riann.h"
#include "riann_internal.h"

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace riann;

struct riann_index {
    riann_params_t prm{};
    int D = 0, Dp = 0, K = 0;
    int64_t n = 0, n_pad = 0;
    std::atomic<int64_t> threshold{0};
    std::atomic<int32_t> shape{0};   // row-layout dense block shape: waves << 8 | cols, 0 = default
    bool dense_rows = true;   // row-layout dense search where supported
    int device = 0;
    // host copies (kept for riann_save)
    std::vector<uint8_t> ref;
    std::vector<int32_t> keys;
    std::vector<uint32_t> T;
    std::vector<int32_t> P;
    std::vector<uint32_t> Piv;
    // device
    void *dmem = nullptr;
    DevIndex dix{};
    unsigned long long *dstats = nullptr;
    std::atomic<uint64_t> frames{0}, full_queries{0};
    std::mutex mu;
    std::map<hipStream_t, Work> work;
    std::map<hipStream_t, std::pair<double *, int64_t>> recon_scratch;  // partials, blocks
    void *paper_mem = nullptr;   // Dm | T | P of the paper's search, n x n each
    std::mutex paper_mu;
    // kernel timing (riann_set_profiling)
    std::atomic<int> profiling{0};   // 0, RIANN_PROFILE_ALL or RIANN_PROFILE_DENSE
    std::mutex pmu;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> evpool;  // read events, ready to be recorded again
    uint64_t prof_launches[RIANN_K_COUNT] = {};
    double prof_ms[RIANN_K_COUNT] = {};
};

// Scratch of riann_match_frame_noalloc: one copy per device, held from the
// library's load until the process ends.  Host code must never pass the
// array's name to a kernel (on the host it is only a stand-in): the device
// address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoAllocScratchBytes = (int64_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err;

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;   // device -> address of its `scratch`

riann_status_t fail(riann_status_t st, const std::string &msg) {
    g_err = msg;
    return st;
}

riann_status_t hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return RIANN_E_DEVICE;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

riann_status_t check_params(const riann_params_t *p) {
    if (!p) return fail(RIANN_E_INVALID, "params is NULL");
    if (p->patch < 1 || p->channels < 1 || p->stride < 1)
        return fail(RIANN_E_INVALID, "patch, channels and stride must be >= 1");
    const int64_t D = (int64_t)p->patch * p->patch * p->channels;
    if (D > 256) return fail(RIANN_E_UNSUPPORTED, "patch dimension p*p*C must be <= 256");
    // the extraction kernel stages a (kExtTY - 1)s + p by (kExtTX - 1)s + p pixel window
    // (rows padded to whole words, plus one spare word) in 64 KB of LDS
    if ((int64_t)((kExtTY - 1) * (int64_t)p->stride + p->patch) *
                ((((kExtTX - 1) * (int64_t)p->stride + p->patch) * p->channels + 3) & ~3) +
            4 > 65536)
        return fail(RIANN_E_UNSUPPORTED, "stride too large for the extraction tile");
    if (p->n_ref < 1 || p->n_ref > (int64_t)0x7FFFFF00)
        return fail(RIANN_E_INVALID, "n_ref must be in [1, 2^31 - 256]");
    if (p->n_keys < 0 || p->n_keys > kMaxKeys)
        return fail(RIANN_E_INVALID, "n_keys must be in [0, 64]");
    if (p->n_keys > p->n_ref) return fail(RIANN_E_INVALID, "n_keys exceeds n_ref");
    if ((p->flags & ~(RIANN_FLAG_COLUMN_DENSE | RIANN_FLAG_EXACT_MSTAR |
                      RIANN_FLAG_GATHER_SCAN)) != 0 ||
        p->reserved != 0)
        return fail(RIANN_E_INVALID, "unknown flags or nonzero reserved field");
    return RIANN_OK;
}

int64_t default_threshold(int64_t n) {
    // ring scan while the smallest ring is below ~1/16 of the set: a scanned
    // candidate costs about 16x a dense (query, reference) pair
    int64_t t = n / 16;
    return t < 64 ? 64 : t;
}

// Rows of the row-layout dense search's reference order (even Rc, then odd
// Rc, each class padded to whole tiles, the whole to kRowAlign).  With
// Rc == nullptr: the most rows any reference set of this size can take.
int64_t row_layout_rows(int64_t n, const std::vector<int32_t> *Rc) {
    int64_t n0 = n;
    if (Rc) {
        n0 = 0;
        for (int64_t r = 0; r < n; ++r) n0 += ((*Rc)[(size_t)r] & 1) == 0;
    }
    return Rc ? round_up(round_up(n0, kTile) + round_up(n - n0, kTile), kRowAlign)
              : round_up(round_up(n, kTile) + kTile, kRowAlign);
}

int64_t index_bytes(int64_t n, int D, int K, uint32_t flags) {
    const int Dp = (int)round_up(D, 32);
    const int64_t n_pad = round_up(n, kRefAlign);
    const int64_t n16 = round_up(n, 16), Kp = round_up(std::max(K, 1), 4);
    const int64_t n_rows = row_layout_rows(n, nullptr);
    const int64_t pivr = (K > 0 && !(flags & RIANN_FLAG_GATHER_SCAN))
                             ? (int64_t)K * n16 * pivr_words(K) * 4 + 256 : 0;
    return 2 * (n_pad * Dp + n_pad * 4) + n_pad * 4 + (int64_t)K * (n16 + n) * 4 + n * Kp * 4 +
           n_rows * ((int64_t)Dp + 12) + (int64_t)K * 4 + (int64_t)kStatWords * 8 + 65536 + 4096 + pivr +
           (int64_t)std::max(K, 1) * kRouteStride * 4 + 256;
}

int64_t work_bytes(int64_t Q, int Dp) { return Q * ((int64_t)Dp + 4 + 1 + 1 + 64 + 8) + 8192; }

// host pre-processing: pivot table and sorted per-key lists
void build_tables(riann_index *h) {
    const int64_t n = h->n;
    const int D = h->D, K = h->K;
    h->Piv.assign((size_t)n * std::max(K, 1), 0);
    h->T.assign((size_t)K * n, 0);
    h->P.assign((size_t)K * n, 0);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto piv_rows = [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r) {
            const uint8_t *a = &h->ref[(size_t)r * D];
            for (int k = 0; k < K; ++k) {
                const uint8_t *b = &h->ref[(size_t)h->keys[k] * D];
                uint32_t s = 0;
                for (int i = 0; i < D; ++i) {
                    int d = (int)a[i] - (int)b[i];
                    s += (uint32_t)(d * d);
                }
                h->Piv[(size_t)r * K + k] = s;
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back(piv_rows, n * t / nt, n * (t + 1) / nt);
    for (auto &x : th) x.join();
    th.clear();
    auto sort_keys = [&](int k0, int k1) {
        std::vector<int32_t> idx((size_t)n);
        for (int k = k0; k < k1; ++k) {
            for (int64_t r = 0; r < n; ++r) idx[(size_t)r] = (int32_t)r;
            std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
                return h->Piv[(size_t)x * K + k] < h->Piv[(size_t)y * K + k];
            });
            for (int64_t j = 0; j < n; ++j) {
                h->P[(size_t)k * n + j] = idx[(size_t)j];
                h->T[(size_t)k * n + j] = h->Piv[(size_t)idx[(size_t)j] * K + k];
            }
        }
    };
    for (unsigned t = 0; t < nt && (int)t < K; ++t)
        th.emplace_back(sort_keys, (int)(K * (int64_t)t / std::min<int64_t>(nt, K)),
                        (int)(K * (int64_t)(t + 1) / std::min<int64_t>(nt, K)));
    for (auto &x : th) x.join();
}

// device upload of everything an index needs
riann_status_t upload(riann_index *h, hipStream_t st) {
    const int64_t n = h->n, n_pad = h->n_pad;
    const int D = h->D, Dp = h->Dp, K = h->K;
    // dense key layout: X = SSD - Qc + bias < 2^(32 - jb) - 1 for every pair
    const int64_t bias = (int64_t)D * 16384;
    const int64_t xmax = (int64_t)D * 65025 + bias;
    int xbits = 1;
    while (((int64_t)1 << xbits) < xmax + 2) ++xbits;
    const int jb = 32 - xbits;
    std::vector<int8_t> Rv((size_t)n_pad * Dp, 0), Rf((size_t)n_pad * Dp, 0);
    std::vector<int32_t> Rc((size_t)n_pad, 0);
    std::vector<uint32_t> Rk((size_t)n_pad, (uint32_t)(((uint64_t)1 << 32) - ((uint64_t)1 << jb)));
    for (int64_t r = 0; r < n; ++r) {
        int32_t s = 0;
        for (int i = 0; i < D; ++i) {
            const int v = (int)h->ref[(size_t)r * D + i] - 128;
            Rv[(size_t)r * Dp + i] = (int8_t)v;
            s += v * (v + 2);
        }
        Rc[(size_t)r] = s;
        Rk[(size_t)r] = (uint32_t)(s + bias) << jb;
    }
    const int KB = Dp / 32;
    for (int64_t r = 0; r < n_pad; ++r)
        for (int kb = 0; kb < KB; ++kb)
            for (int g = 0; g < 2; ++g) {
                const int64_t t = r / kTile, l = (r % kTile) + 32 * g;
                std::memcpy(&Rf[(size_t)(((t * KB + kb) * 64 + l) * 16)],
                            &Rv[(size_t)(r * Dp + kb * 32 + 16 * g)], 16);
            }
    // row-layout tables over the class order (even Rc, then odd Rc)
    const int64_t n_rows = row_layout_rows(n, &Rc);
    std::vector<int8_t> Rfr((size_t)n_rows * Dp, 0);
    std::vector<int32_t> Hf((size_t)n_rows, row_pad_y(Dp));
    std::vector<int32_t> Rci((size_t)n_rows * 2, 0);
    {
        std::vector<int64_t> order((size_t)n_rows, -1);
        int64_t pos = 0;
        for (int cls = 0; cls < 2; ++cls) {
            for (int64_t r = 0; r < n; ++r)
                if ((Rc[(size_t)r] & 1) == cls) order[(size_t)pos++] = r;
            pos = round_up(pos, kTile);
        }
        for (int64_t i = 0; i < n_rows; ++i) {
            const int64_t r = order[(size_t)i];
            Rci[(size_t)(2 * i)] = r < 0 ? 0 : Rc[(size_t)r];
            Rci[(size_t)(2 * i + 1)] = (int32_t)r;
            if (r < 0) continue;
            const int64_t t = i / kTile;
            for (int kb = 0; kb < KB; ++kb)
                for (int g = 0; g < 2; ++g)
                    std::memcpy(&Rfr[(size_t)(((t * KB + kb) * 64 + (i % kTile) + 32 * g) * 16)],
                                &Rv[(size_t)(r * Dp + kb * 32 + 16 * g)], 16);
        }
        for (int64_t t = 0; t < n_rows / kTile; ++t)
            for (int g = 0; g < 2; ++g)
                for (int r = 0; r < 16; ++r) {
                    // accumulator order: entry g * 16 + r of a tile is row 8(r/4) + 4g + r%4
                    const int64_t ref = order[(size_t)(t * kTile + 8 * (r / 4) + 4 * g + r % 4)];
                    if (ref < 0) continue;
                    const int64_t rc = Rc[(size_t)ref];
                    Hf[(size_t)(t * kTile + g * 16 + r)] = (int32_t)((rc + bias - (rc & 1)) / 2);
                }
    }
    // ring-phase tables: T padded to 16-entry lines, LDS samples, padded Piv
    const int64_t n16 = round_up(n, 16);
    // ring-size lower bounds: per key, B value buckets of width 2^shift from
    // the key's smallest distance vmin, and cdf[j] = #{entries < vmin +
    // j 2^shift}, j = 0..B; row k = {vmin, shift, cdf[0..B]} padded to lbS
    const int lbB = lb_buckets(K), lbS = lb_stride(K);
    std::vector<uint32_t> Lb((size_t)std::max(K, 1) * lbS, 0u);
    for (int k = 0; k < K; ++k) {
        const uint32_t *t = &h->T[(size_t)k * n];
        const uint64_t vmin = t[0], vmax = t[n - 1];
        int sh = 0;
        while (((vmax - vmin) >> sh) >= (uint64_t)lbB) ++sh;
        uint32_t *row = &Lb[(size_t)k * lbS];
        row[0] = (uint32_t)vmin;
        row[1] = (uint32_t)sh;
        for (int j = 0; j <= lbB; ++j) {
            const uint64_t edge = vmin + ((uint64_t)j << sh);
            row[2 + j] = (uint32_t)(std::lower_bound(t, t + n, edge,
                                                     [](uint32_t x, uint64_t e) { return x < e; }) - t);
        }
    }
    // routing rows in square-root space (the extraction kernel's test): per
    // key, origin o = floor(sqrt(vmin)) and bucket width 2^e, the smallest
    // with o + B 2^e > sqrt(vmax) (e >= -16); F[j] = #{entries a :
    // sqrt(a) < x_j}, x_j = o + j 2^e, i.e. entries below ceil(x_j^2), which
    // integer arithmetic gives exactly
    std::vector<uint32_t> Rt((size_t)std::max(K, 1) * kRouteStride, 0u);
    for (int k = 0; k < K; ++k) {
        const uint32_t *t = &h->T[(size_t)k * n];
        const uint64_t vmin = t[0], vmax = t[n - 1];
        uint64_t o = (uint64_t)std::sqrt((double)vmin);
        while (o * o > vmin) --o;
        while ((o + 1) * (o + 1) <= vmin) ++o;
        // x_j^2 > a for every entry once x_j^2 > vmax
        auto above_max = [&](int e, uint64_t j) {
            if (e >= 0) {
                const uint64_t x = o + (j << e);
                return x * x > vmax;
            }
            const uint64_t m = 1ull << (-e), x = o * m + j;   // x_j = x / m
            return x * x > vmax * m * m;
        };
        int e = -16;
        while (!above_max(e, kRouteBuckets)) ++e;
        uint32_t *row = &Rt[(size_t)k * kRouteStride];
        const float of = (float)o, inv = std::ldexp(1.0f, -e);
        std::memcpy(&row[0], &of, 4);
        std::memcpy(&row[1], &inv, 4);
        for (int j = 0; j <= kRouteBuckets; ++j) {
            uint64_t c2;   // ceil(x_j^2)
            if (e >= 0) {
                const uint64_t x = o + ((uint64_t)j << e);
                c2 = x * x;
            } else {
                const uint64_t m = 1ull << (-e), x = o * m + (uint64_t)j, d = m * m;
                c2 = (x * x + d - 1) / d;
            }
            row[2 + j] = (uint32_t)(std::lower_bound(t, t + n, c2,
                                                     [](uint32_t a, uint64_t v) { return a < v; }) - t);
        }
    }
    int64_t s0l = 1;   // sample stride in lines: samples, bound rows, key rows and
                       // key Rc of all keys fit 64 KB of LDS
    while ((int64_t)K * (((n + 16 * s0l - 1) / (16 * s0l) + 3) / 4 * 4 + lbS + Dp / 4 + 1) * 4 >
           65536)
        s0l *= 2;
    const int64_t ns = (n + 16 * s0l - 1) / (16 * s0l);
    const int Kp = (int)round_up(std::max(K, 1), 4);
    std::vector<uint32_t> Tl((size_t)K * n16, 0xFFFFFFFFu), Ts((size_t)std::max<int64_t>(K * ns, 1));
    std::vector<uint32_t> Pv((size_t)n * Kp, 0u);
    for (int k = 0; k < K; ++k) {
        std::memcpy(&Tl[(size_t)k * n16], &h->T[(size_t)k * n], (size_t)n * 4);
        for (int64_t i = 0; i < ns; ++i) Ts[(size_t)(k * ns + i)] = h->T[(size_t)(k * n + i * 16 * s0l)];
    }
    for (int64_t r = 0; r < n; ++r)
        for (int k = 0; k < K; ++k) Pv[(size_t)(r * Kp + k)] = h->Piv[(size_t)(r * K + k)];
    const size_t szRv = (size_t)n_pad * Dp, szRc = (size_t)n_pad * 4,
                 szT = (size_t)std::max<int64_t>(K * n16, 1) * 4,
                 szP = (size_t)std::max<int64_t>(K * n, 1) * 4,
                 szPiv = (size_t)n * Kp * 4, szK = (size_t)std::max(K, 1) * 4,
                 szS = (size_t)kStatWords * 8, szTs = Ts.size() * 4, szLb = Lb.size() * 4;
    const size_t szRfr = (size_t)n_rows * Dp, szHf = (size_t)n_rows * 4, szRci = (size_t)n_rows * 8;
    const bool pivr = K > 0 && !(h->prm.flags & RIANN_FLAG_GATHER_SCAN);
    const size_t szPivR = pivr ? (size_t)K * n16 * pivr_words(K) * 4 : 0;
    const size_t szRt = Rt.size() * 4;
    size_t off[16], tot = 0;
    const size_t sz[16] = {szRv, szRc, szT, szP, szPiv, szK, szS, szRv, szRc, szTs, szHf, szRfr, szRci,
                           szLb, szPivR, szRt};
    for (int i = 0; i < 16; ++i) {
        off[i] = tot;
        tot += round_up((int64_t)sz[i], 256);
    }
    hipError_t e = hipMalloc(&h->dmem, tot);
    if (e != hipSuccess) {
        h->dmem = nullptr;
        return fail(RIANN_E_NOMEM, std::string("hipMalloc of the index failed: ") +
                                       hipGetErrorString(e));
    }
    char *b = (char *)h->dmem;
    h->dix.Rv = (const int8_t *)(b + off[0]);
    h->dix.Rc = (const int32_t *)(b + off[1]);
    h->dix.T = (const uint32_t *)(b + off[2]);
    h->dix.P = (const int32_t *)(b + off[3]);
    h->dix.Piv = (const uint32_t *)(b + off[4]);
    h->dix.keys = (const int32_t *)(b + off[5]);
    h->dstats = (unsigned long long *)(b + off[6]);
    h->dix.Rf = (const int8_t *)(b + off[7]);
    h->dix.Rk = (const uint32_t *)(b + off[8]);
    h->dix.jb = jb;
    h->dix.bias = (int32_t)bias;
    h->dix.Ts = (const uint32_t *)(b + off[9]);
    h->dix.Lb = (const uint32_t *)(b + off[13]);
    h->dix.lbB = lbB;
    h->dix.lbS = lbS;
    h->dix.exact_mstar = (h->prm.flags & RIANN_FLAG_EXACT_MSTAR) ? 1 : 0;
    h->dix.PivR = pivr ? (const uint32_t *)(b + off[14]) : nullptr;
    h->dix.Rt = (const uint32_t *)(b + off[15]);
    h->dix.rtS = kRouteStride;
    h->dix.KR = pivr ? pivr_words(K) : 0;
    h->dix.Hf = (const int32_t *)(b + off[10]);
    h->dix.Rfr = (const int8_t *)(b + off[11]);
    h->dix.Rci = (const int2 *)(b + off[12]);
    h->dix.n_rows = n_rows;
    h->dix.n16 = (int32_t)n16;
    h->dix.ns = (int32_t)ns;
    h->dix.s0l = (int32_t)s0l;
    h->dix.Kp = Kp;
    h->dix.n = n;
    h->dix.n_pad = n_pad;
    h->dix.D = D;
    h->dix.Dp = Dp;
    h->dix.K = K;
    h->dix.p = h->prm.patch;
    h->dix.C = h->prm.channels;
    h->dix.s = h->prm.stride;
    struct { void *dst; const void *src; size_t n; } cp[] = {
        {b + off[0], Rv.data(), szRv},          {b + off[1], Rc.data(), szRc},
        {b + off[2], Tl.data(), (size_t)K * n16 * 4}, {b + off[3], h->P.data(), (size_t)K * n * 4},
        {b + off[4], Pv.data(), szPiv},
        {b + off[5], h->keys.data(), (size_t)K * 4},
        {b + off[7], Rf.data(), szRv},          {b + off[8], Rk.data(), szRc},
        {b + off[9], Ts.data(), (size_t)K * ns * 4},
        {b + off[13], Lb.data(), szLb},
        {b + off[15], Rt.data(), szRt},
        {b + off[10], Hf.data(), szHf},
        {b + off[11], Rfr.data(), szRfr},
        {b + off[12], Rci.data(), szRci},
    };
    for (auto &c : cp) {
        if (c.n == 0) continue;
        e = hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "index upload");
    }
    e = hipMemsetAsync(h->dstats, 0, szS, st);
    if (e != hipSuccess) return hip_fail(e, "stats clear");
    if (pivr) {
        // ring-ordered pivot rows, gathered on the device from P and Piv
        e = launch_build_pivr(h->dix, (uint32_t *)(b + off[14]), st);
        if (e != hipSuccess) return hip_fail(e, "pivot-row table build");
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "index upload sync");
    return RIANN_OK;
}

void free_index(riann_index *h) {
    if (!h) return;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (auto &p : h->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
    for (auto &kv : h->work) (void)hipFree(kv.second.patches);
    for (auto &kv : h->recon_scratch) (void)hipFree(kv.second.first);
    if (h->paper_mem) (void)hipFree(h->paper_mem);
    if (h->dmem) (void)hipFree(h->dmem);
    delete h;
}

riann_status_t finish_build(riann_index *h, hipStream_t st, riann_index_t *out) {
    riann_status_t s = upload(h, st);
    if (s != RIANN_OK) {
        free_index(h);
        return s;
    }
    *out = h;
    return RIANN_OK;
}

// The per-launch scratch of `cap` queries laid out from `b` (work_bytes(cap,
// Dp) bytes, 256-byte aligned).
Work carve_work(char *b, int64_t cap, int Dp) {
    Work nw;
    int64_t o = 0;
    nw.patches = (uint8_t *)(b + o);  o = round_up(o + cap * Dp, 256);
    nw.qc = (int32_t *)(b + o);       o = round_up(o + cap * 4, 256);
    nw.fid = (uint8_t *)(b + o);      o = round_up(o + cap, 256);
    nw.route = (uint8_t *)(b + o);    o = round_up(o + cap, 256);
    nw.rec = (uint4 *)(b + o);        o = round_up(o + cap * 16, 256);
    nw.rec2 = (uint4 *)(b + o);       o = round_up(o + cap * 48, 256);
    nw.ring_list = (uint32_t *)(b + o); o = round_up(o + cap * 4, 256);
    nw.dense_list = (uint32_t *)(b + o); o = round_up(o + cap * 4, 256);
    nw.counters = (uint32_t *)(b + o);
    nw.capacity = cap;
    return nw;
}

riann_status_t get_work(riann_index *h, hipStream_t st, int64_t Q, Work *w) {
    const int Dp = h->Dp;
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->work.find(st);
    if (it != h->work.end() && it->second.capacity >= Q) {
        *w = it->second;
        return RIANN_OK;
    }
    if (it != h->work.end()) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "scratch resize sync");
        (void)hipFree(it->second.patches);
        h->work.erase(it);
    }
    const int64_t cap = std::max<int64_t>(Q, 4096);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)work_bytes(cap, Dp));
    if (e != hipSuccess) return fail(RIANN_E_NOMEM, "hipMalloc of frame scratch failed");
    const Work nw = carve_work((char *)p, cap, Dp);
    h->work[st] = nw;
    *w = nw;
    return RIANN_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b) return false;
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// Checks one frame and fills its descriptor (qbase/tbase are set later).
riann_status_t frame_desc(const riann_index *h, const uint8_t *frame, int32_t H, int32_t W,
                          int64_t pitch, const int32_t *prev, int32_t *out, uint32_t *ssd,
                          int32_t mode, FrameDesc *fd, int knn = 1) {
    const int p = h->prm.patch, C = h->prm.channels, s = h->prm.stride;
    if (!frame) return fail(RIANN_E_INVALID, "frame is NULL");
    if (!out) return fail(RIANN_E_INVALID, "out is NULL");
    if (mode != RIANN_MODE_RING && mode != RIANN_MODE_FULL)
        return fail(RIANN_E_INVALID, "bad frame mode");
    if (H < p || W < p) return fail(RIANN_E_INVALID, "frame smaller than one patch");
    if (pitch < (int64_t)W * C) return fail(RIANN_E_INVALID, "pitch < W * channels");
    fd->frame = frame;
    fd->pitch = pitch;
    fd->H = H;
    fd->W = W;
    fd->Hq = (H - p) / s + 1;
    fd->Wq = (W - p) / s + 1;
    fd->mode = mode;
    fd->prev = mode == RIANN_MODE_RING ? prev : nullptr;
    fd->out = out;
    fd->ssd = ssd;
    const int64_t Q = (int64_t)fd->Hq * fd->Wq;
    if (Q >= (int64_t)0x7FFFFFFF) return fail(RIANN_E_UNSUPPORTED, "too many queries in one frame");
    const size_t qb = (size_t)Q * 4 * knn;
    if (overlap(fd->prev, qb, out, qb)) return fail(RIANN_E_INVALID, "prev overlaps out");
    if (overlap(ssd, qb, out, qb)) return fail(RIANN_E_INVALID, "ssd overlaps out");
    if (overlap(fd->prev, qb, ssd, qb)) return fail(RIANN_E_INVALID, "prev overlaps ssd");
    return RIANN_OK;
}

// Records a start event when profiling is on; the matching stop() records
// the end event and queues the pair for riann_get_profile.
struct KTimer {
    riann_index *h;
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr;
    KTimer(riann_index *h_, int kind_, hipStream_t st_, bool on = true)
        : h(h_), kind(kind_), st(st_) {
        const int lv = on ? h->profiling.load() : 0;
        if (lv == 0) return;
        if (lv == RIANN_PROFILE_DENSE && kind != RIANN_K_DENSE && kind != RIANN_K_FULL) return;
        a = take();
        if (a) (void)hipEventRecord(a, st);
    }
    hipEvent_t take() {
        {
            std::lock_guard<std::mutex> lk(h->pmu);
            if (!h->evpool.empty()) {
                hipEvent_t e = h->evpool.back();
                h->evpool.pop_back();
                return e;
            }
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    void stop() {
        if (!a) return;
        hipEvent_t b = take();
        std::lock_guard<std::mutex> lk(h->pmu);
        if (!b) {
            h->evpool.push_back(a);
        } else {
            (void)hipEventRecord(b, st);
            h->pending.push_back({kind, a, b});
        }
        a = nullptr;
    }
};

// One launch sequence over up to kMaxBatch frames (descriptors validated).
// `preset`: scratch the caller provides (the no-allocation entry point); then
// nothing is allocated and no profiling events are taken.
riann_status_t run_batch(riann_index *h, FrameBatch &fb, hipStream_t st, int knn = 1,
                         const Work *preset = nullptr) {
    fb.knn = knn;
    fb.dense_masked = 0;
    int64_t q = 0;
    int32_t t = 0;
    bool all_full = true;
    for (int i = 0; i < fb.n; ++i) {
        FrameDesc &fd = fb.f[i];
        fd.qbase = q;
        fd.tbase = t;
        q += (int64_t)fd.Hq * fd.Wq;
        t += ((fd.Wq + kExtTX - 1) / kExtTX) * ((fd.Hq + kExtTY - 1) / kExtTY);
        all_full = all_full && fd.mode == RIANN_MODE_FULL;
    }
    if (q >= (int64_t)0x7FFFFFFF) return fail(RIANN_E_UNSUPPORTED, "too many queries in one batch");
    fb.Q = q;
    fb.ntiles = t;
    fb.all_full = all_full ? 1 : 0;
    Work w;
    if (preset) {
        if (preset->capacity < q) return fail(RIANN_E_INVALID, "scratch smaller than the batch");
        w = *preset;
    } else {
        riann_status_t s = get_work(h, st, q, &w);
        if (s != RIANN_OK) return s;
    }
    hipError_t e;
    const bool rows = knn == 1 && h->dense_rows && dense_rows_supported(h->dix);
    // the row-layout search takes the queries in order and skips the
    // ring-scanned ones by their route codes: no dense list is built
    fb.dense_masked = rows && !all_full ? kDenseMasked : 0;
    const bool timed = preset == nullptr;
    // one threshold for the whole launch: the extraction kernel routes on it
    // and the ring kernel decides the rest with it
    const int64_t threshold = h->threshold.load();
    // With route codes and a threshold below 1 the extraction kernel sends
    // every query to the dense search (m* >= 1 by containment): the ring
    // kernel would find nothing to do
    const bool ring_empty = fb.dense_masked && knn == 1 && h->dix.K > 0 &&
                            !h->dix.exact_mstar && threshold >= 0 && threshold < 1;
    // One frame whose every query goes dense, of a shape the dense search can
    // cut from the frame itself: no extraction launch (the dense kernel also
    // counts a ring frame's routing)
    fb.fused = rows && fb.n == 1 && (all_full || ring_empty) && dense_fused_supported(h->dix)
                   ? 1 : 0;
    fb.stats = h->dstats;
    if (!fb.fused) {
        // the extraction kernel also clears the ring and dense list counters
        KTimer tm(h, RIANN_K_EXTRACT, st, timed);
        e = launch_extract(h->dix, fb, w, threshold, h->dstats, st);
        tm.stop();
        if (e != hipSuccess) return hip_fail(e, "k_extract launch");
    }
    if (!all_full && !ring_empty) {
        {
            KTimer tm(h, RIANN_K_RING, st, timed);
            e = launch_ring(h->dix, fb, w, h->dstats, threshold, st);
            tm.stop();
            if (e != hipSuccess) return hip_fail(e, "k_ring launch");
        }
        if (!ring_scans_inline(h->dix, fb)) {
            KTimer tm(h, RIANN_K_SCAN, st, timed);
            e = knn > 1 ? launch_scan_knn(h->dix, fb, w, h->dstats, st)
                        : launch_scan(h->dix, fb, w, h->dstats, st);
            tm.stop();
            if (e != hipSuccess) return hip_fail(e, "k_scan launch");
        }
    }
    // nothing was ring-scanned: the dense search takes every query in order
    // without reading the route codes, as a full search does
    if (ring_empty) fb.dense_masked = kDenseInOrder;
    {
        KTimer tm(h, all_full ? RIANN_K_FULL : RIANN_K_DENSE, st, timed);
        if (knn > 1) {
            e = h->dense_rows && knn_rows_supported(h->dix) ? launch_dense_rows_knn(h->dix, fb, w, st)
                                                            : launch_dense_knn(h->dix, fb, w, st);
        } else if (rows) {
            DevIndex dx = h->dix;
            const int32_t sh = h->shape.load();
            dx.row_waves = sh >> 8;
            dx.row_cols = sh & 0xFF;
            e = launch_dense_rows(dx, fb, w, st);
        } else {
            e = launch_dense(h->dix, fb, w, st);
        }
        tm.stop();
        if (e != hipSuccess) return hip_fail(e, "k_dense launch");
    }
    h->frames.fetch_add((uint64_t)fb.n);
    if (all_full) h->full_queries.fetch_add((uint64_t)q);
    return RIANN_OK;
}

const char kMagic[8] = {'R', 'I', 'A', 'N', 'N', 'I', 'D', 'X'};
const uint32_t kFileVersion = 1;

}  // namespace

extern "C" {

uint32_t riann_version(void) { return (1u << 16) | 1u; }

const char *riann_last_error(void) { return g_err.c_str(); }

riann_status_t riann_footprint(const riann_params_t *p, int32_t H, int32_t W, int64_t *bytes) {
    riann_status_t s = check_params(p);
    if (s != RIANN_OK) return s;
    if (!bytes) return fail(RIANN_E_INVALID, "bytes is NULL");
    int64_t b = index_bytes(p->n_ref, p->patch * p->patch * p->channels, p->n_keys, p->flags);
    if (H > 0 && W > 0) {
        if (H < p->patch || W < p->patch) return fail(RIANN_E_INVALID, "frame smaller than patch");
        const int64_t Q = (int64_t)((H - p->patch) / p->stride + 1) *
                          ((W - p->patch) / p->stride + 1);
        b += work_bytes(std::max<int64_t>(Q, 4096),
                        (int)round_up((int64_t)p->patch * p->patch * p->channels, 32));
    }
    *bytes = b;
    return RIANN_OK;
}

riann_status_t riann_build(const uint8_t *ref_host, const int32_t *key_idx,
                           const riann_params_t *p, void *hip_stream, riann_index_t *out) {
    riann_status_t s = check_params(p);
    if (s != RIANN_OK) return s;
    if (!ref_host || !out) return fail(RIANN_E_INVALID, "ref or out is NULL");
    if (p->n_keys > 0 && !key_idx) return fail(RIANN_E_INVALID, "key_idx is NULL");
    std::vector<char> seen((size_t)p->n_ref, 0);
    for (int k = 0; k < p->n_keys; ++k) {
        const int32_t v = key_idx[k];
        if (v < 0 || (int64_t)v >= p->n_ref) return fail(RIANN_E_INVALID, "key index out of range");
        if (seen[(size_t)v]) return fail(RIANN_E_INVALID, "duplicate key index");
        seen[(size_t)v] = 1;
    }
    riann_index *h = new (std::nothrow) riann_index();
    if (!h) return fail(RIANN_E_NOMEM, "host allocation failed");
    h->prm = *p;
    h->D = p->patch * p->patch * p->channels;
    h->Dp = (int)round_up(h->D, 32);
    h->K = p->n_keys;
    h->n = p->n_ref;
    h->n_pad = round_up(h->n, kRefAlign);
    h->dense_rows = (p->flags & RIANN_FLAG_COLUMN_DENSE) == 0;
    h->threshold.store(p->dense_threshold >= 0 ? p->dense_threshold : default_threshold(h->n));
    h->prm.dense_threshold = h->threshold.load();
    (void)hipGetDevice(&h->device);
    try {
        h->ref.assign(ref_host, ref_host + (size_t)h->n * h->D);
        h->keys.assign(key_idx, key_idx + h->K);
        build_tables(h);
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(RIANN_E_NOMEM, "host allocation failed");
    }
    return finish_build(h, (hipStream_t)hip_stream, out);
}

riann_status_t riann_match_frame(riann_index_t h, const uint8_t *frame_dev, int32_t H, int32_t W,
                                 int64_t pitch, const int32_t *prev_dev, int32_t *out_dev,
                                 uint32_t *ssd_dev, void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    FrameBatch fb;
    fb.n = 1;
    riann_status_t s = frame_desc(h, frame_dev, H, W, pitch, prev_dev, out_dev, ssd_dev,
                                  RIANN_MODE_RING, &fb.f[0]);
    if (s != RIANN_OK) return s;
    DeviceGuard g(h->device);
    return run_batch(h, fb, (hipStream_t)hip_stream);
}

riann_status_t riann_match_frame_noalloc(riann_index_t h, const uint8_t *frame_dev, int32_t H,
                                         int32_t W, int64_t pitch, const int32_t *prev_dev,
                                         int32_t *out_dev, uint32_t *ssd_dev, void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    FrameBatch fb;
    fb.n = 1;
    riann_status_t s = frame_desc(h, frame_dev, H, W, pitch, prev_dev, out_dev, ssd_dev,
                                  RIANN_MODE_RING, &fb.f[0]);
    if (s != RIANN_OK) return s;
    const int64_t Q = (int64_t)fb.f[0].Hq * fb.f[0].Wq;
    const int64_t need = work_bytes(Q, h->Dp);
    if (need > kNoAllocScratchBytes)
        return fail(RIANN_E_UNSUPPORTED,
                    "frame of " + std::to_string(Q) + " queries needs " + std::to_string(need) +
                        " bytes of scratch, more than the " +
                        std::to_string(kNoAllocScratchBytes) +
                        " bytes riann_match_frame_noalloc holds");
    DeviceGuard g(h->device);
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch_ptr.find(h->device);
        if (it == g_scratch_ptr.end()) {
            void *ptr = nullptr;
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return hip_fail(e, "scratch symbol address");
            it = g_scratch_ptr.emplace(h->device, (char *)ptr).first;
        }
        base = it->second;
    }
    // every buffer that must start at zero (the list counters) is cleared by
    // the extraction kernel of the launch itself
    const Work w = carve_work(base, Q, h->Dp);
    return run_batch(h, fb, (hipStream_t)hip_stream, 1, &w);
}

riann_status_t riann_match_knn(riann_index_t h, const uint8_t *frame_dev, int32_t H, int32_t W,
                               int64_t pitch, int32_t k, const int32_t *prev_dev, int32_t *out_dev,
                               uint32_t *ssd_dev, int32_t mode, void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (k < 1 || k > kMaxKnn) return fail(RIANN_E_INVALID, "k must be in [1, 8]");
    if (k > h->n) return fail(RIANN_E_INVALID, "k exceeds the number of references");
    if (k > 1 && !(h->dense_rows && knn_rows_supported(h->dix)) && !knn_dense_supported(h->dix))
        return fail(RIANN_E_UNSUPPORTED,
                    "k-NN fields: reference set too large for this patch size (see riann.h)");
    FrameBatch fb;
    fb.n = 1;
    riann_status_t s = frame_desc(h, frame_dev, H, W, pitch, prev_dev, out_dev, ssd_dev, mode,
                                  &fb.f[0], k);
    if (s != RIANN_OK) return s;
    DeviceGuard g(h->device);
    return run_batch(h, fb, (hipStream_t)hip_stream, k);
}

riann_status_t riann_full_search(riann_index_t h, const uint8_t *frame_dev, int32_t H, int32_t W,
                                 int64_t pitch, int32_t *out_dev, uint32_t *ssd_dev,
                                 void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    FrameBatch fb;
    fb.n = 1;
    riann_status_t s = frame_desc(h, frame_dev, H, W, pitch, nullptr, out_dev, ssd_dev,
                                  RIANN_MODE_FULL, &fb.f[0]);
    if (s != RIANN_OK) return s;
    DeviceGuard g(h->device);
    return run_batch(h, fb, (hipStream_t)hip_stream);
}

riann_status_t riann_match_batch(riann_index_t h, const riann_frame_desc_t *descs, int32_t n,
                                 void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (n < 0 || (n > 0 && !descs)) return fail(RIANN_E_INVALID, "bad descriptor array");
    std::vector<FrameDesc> fds((size_t)n);
    for (int i = 0; i < n; ++i) {
        const riann_frame_desc_t &d = descs[i];
        riann_status_t s = frame_desc(h, d.frame, d.H, d.W, d.pitch, d.prev, d.out, d.ssd, d.mode,
                                      &fds[(size_t)i]);
        if (s != RIANN_OK) return s;
    }
    // outputs of different frames must not overlap
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const size_t qi = (size_t)fds[(size_t)i].Hq * fds[(size_t)i].Wq * 4;
            const size_t qj = (size_t)fds[(size_t)j].Hq * fds[(size_t)j].Wq * 4;
            const FrameDesc &a = fds[(size_t)i], &b = fds[(size_t)j];
            if (overlap(a.out, qi, b.out, qj) || overlap(a.out, qi, b.ssd, qj) ||
                overlap(a.ssd, qi, b.out, qj) || overlap(a.ssd, qi, b.ssd, qj))
                return fail(RIANN_E_INVALID, "output fields of two frames overlap");
        }
    DeviceGuard g(h->device);
    hipStream_t st = (hipStream_t)hip_stream;
    for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
        FrameBatch fb;
        fb.n = std::min(kMaxBatch, n - i0);
        for (int i = 0; i < fb.n; ++i) fb.f[i] = fds[(size_t)(i0 + i)];
        riann_status_t s = run_batch(h, fb, st);
        if (s != RIANN_OK) return s;
    }
    return RIANN_OK;
}

riann_status_t riann_get_stats(riann_index_t h, riann_stats_t *s) {
    if (!h || !s) return fail(RIANN_E_INVALID, "NULL argument");
    DeviceGuard g(h->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device sync");
    std::vector<unsigned long long> rep((size_t)kStatWords);
    e = hipMemcpy(rep.data(), h->dstats, rep.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stats copy");
    unsigned long long v[ST_COUNT] = {};
    for (int slot = 0; slot < ST_COUNT; ++slot)
        for (int r = 0; r < kStatReplicas; ++r)
            v[slot] += rep[((size_t)slot * kStatReplicas + r) * kStatStride];
    const uint64_t fq = h->full_queries.load();
    s->frames = h->frames.load();
    s->queries = v[ST_QUERIES] + fq;
    s->ring_queries = v[ST_RING];
    s->dense_queries = v[ST_DENSE] + fq;
    s->no_prior = v[ST_NOPRIOR];
    s->sum_mstar = v[ST_MSTAR];
    s->sum_survivors = v[ST_SURV];
    s->sum_mstar_ring = v[ST_MSTAR_RING];
    s->bound_routed = v[ST_BOUND];
    s->dense_routed = v[ST_DENSE];
    s->bsearch_probes = v[ST_PROBES];
    return RIANN_OK;
}

riann_status_t riann_reset_stats(riann_index_t h) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    DeviceGuard g(h->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device sync");
    e = hipMemset(h->dstats, 0, (size_t)kStatWords * 8);
    if (e != hipSuccess) return hip_fail(e, "stats clear");
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device sync");
    h->frames.store(0);
    h->full_queries.store(0);
    return RIANN_OK;
}

riann_status_t riann_get_params(riann_index_t h, riann_params_t *p) {
    if (!h || !p) return fail(RIANN_E_INVALID, "NULL argument");
    *p = h->prm;
    return RIANN_OK;
}

riann_status_t riann_set_dense_threshold(riann_index_t h, int64_t threshold) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (threshold < 0) return fail(RIANN_E_INVALID, "threshold must be >= 0");
    h->threshold.store(threshold);
    h->prm.dense_threshold = threshold;
    return RIANN_OK;
}

riann_status_t riann_set_dense_shape(riann_index_t h, int32_t waves, int32_t cols) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (waves == 0 && cols == 0) {
        h->shape.store(0);
        return RIANN_OK;
    }
    if (!h->dense_rows) return fail(RIANN_E_UNSUPPORTED, "the column-layout dense search has one shape");
    int32_t wv[16], cl[16];
    const int n = dense_rows_shapes(h->Dp, wv, cl, 16);
    for (int i = 0; i < n && i < 16; ++i)
        if (wv[i] == waves && cl[i] == cols) {
            h->shape.store(i == 0 ? 0 : (waves << 8 | cols));
            return RIANN_OK;
        }
    return fail(RIANN_E_UNSUPPORTED, "block shape " + std::to_string(waves) + " x " +
                                         std::to_string(cols) + " is not built for this patch width");
}

riann_status_t riann_get_dense_shapes(riann_index_t h, int32_t *waves, int32_t *cols, int32_t max,
                                      int32_t *count, int32_t *current) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (max < 0) return fail(RIANN_E_INVALID, "max must be >= 0");
    int32_t wv[16], cl[16];
    const int n = h->dense_rows ? std::min(dense_rows_shapes(h->Dp, wv, cl, 16), 16) : 0;
    const int32_t sh = h->shape.load();
    int cur = 0;
    for (int i = 0; i < n; ++i) {
        if (i < max) {
            if (waves) waves[i] = wv[i];
            if (cols) cols[i] = cl[i];
        }
        if (sh != 0 && (wv[i] << 8 | cl[i]) == sh) cur = i;
    }
    if (count) *count = n;
    if (current) *current = cur;
    return RIANN_OK;
}

riann_status_t riann_save(riann_index_t h, const char *path) {
    if (!h || !path) return fail(RIANN_E_INVALID, "NULL argument");
    {
        DeviceGuard g(h->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "device sync");
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(RIANN_E_IO, std::string("cannot open for writing: ") + path);
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 &&
              std::fwrite(&kFileVersion, 4, 1, f) == 1 &&
              std::fwrite(&h->prm, sizeof(riann_params_t), 1, f) == 1;
    auto put = [&](const void *d, size_t n) {
        if (ok && n) ok = std::fwrite(d, 1, n, f) == n;
    };
    put(h->ref.data(), h->ref.size());
    put(h->keys.data(), h->keys.size() * 4);
    put(h->T.data(), h->T.size() * 4);
    put(h->P.data(), h->P.size() * 4);
    put(h->Piv.data(), (size_t)h->n * h->K * 4);
    if (std::fclose(f) != 0) ok = false;
    if (!ok) return fail(RIANN_E_IO, std::string("write failed: ") + path);
    return RIANN_OK;
}

riann_status_t riann_load(const char *path, void *hip_stream, riann_index_t *out) {
    if (!path || !out) return fail(RIANN_E_INVALID, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(RIANN_E_IO, std::string("cannot open: ") + path);
    char magic[8];
    uint32_t ver = 0;
    riann_params_t prm;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(&ver, 4, 1, f) == 1 && ver == kFileVersion &&
              std::fread(&prm, sizeof(prm), 1, f) == 1;
    if (!ok) {
        std::fclose(f);
        return fail(RIANN_E_IO, "not a riann index file (or wrong version)");
    }
    riann_status_t s = check_params(&prm);
    if (s != RIANN_OK) {
        std::fclose(f);
        return s;
    }
    riann_index *h = new (std::nothrow) riann_index();
    if (!h) {
        std::fclose(f);
        return fail(RIANN_E_NOMEM, "host allocation failed");
    }
    h->prm = prm;
    h->D = prm.patch * prm.patch * prm.channels;
    h->Dp = (int)round_up(h->D, 32);
    h->K = prm.n_keys;
    h->n = prm.n_ref;
    h->n_pad = round_up(h->n, kRefAlign);
    h->dense_rows = (prm.flags & RIANN_FLAG_COLUMN_DENSE) == 0;
    h->threshold.store(prm.dense_threshold >= 0 ? prm.dense_threshold : default_threshold(h->n));
    h->prm.dense_threshold = h->threshold.load();
    (void)hipGetDevice(&h->device);
    try {
        h->ref.resize((size_t)h->n * h->D);
        h->keys.resize((size_t)h->K);
        h->T.resize((size_t)h->K * h->n);
        h->P.resize((size_t)h->K * h->n);
        h->Piv.assign((size_t)h->n * std::max(h->K, 1), 0);
    } catch (const std::bad_alloc &) {
        std::fclose(f);
        delete h;
        return fail(RIANN_E_NOMEM, "host allocation failed");
    }
    auto get = [&](void *d, size_t n) {
        if (ok && n) ok = std::fread(d, 1, n, f) == n;
    };
    get(h->ref.data(), h->ref.size());
    get(h->keys.data(), h->keys.size() * 4);
    get(h->T.data(), h->T.size() * 4);
    get(h->P.data(), h->P.size() * 4);
    get(h->Piv.data(), (size_t)h->n * h->K * 4);
    std::fclose(f);
    if (!ok) {
        delete h;
        return fail(RIANN_E_IO, "truncated index file");
    }
    for (int k = 0; k < h->K; ++k)
        if (h->keys[(size_t)k] < 0 || h->keys[(size_t)k] >= h->n) {
            delete h;
            return fail(RIANN_E_IO, "corrupt key index in file");
        }
    for (size_t i = 0; i < h->P.size(); ++i)
        if (h->P[i] < 0 || h->P[i] >= h->n) {
            delete h;
            return fail(RIANN_E_IO, "corrupt table in file");
        }
    return finish_build(h, (hipStream_t)hip_stream, out);
}

riann_status_t riann_set_profiling(riann_index_t h, int enable) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (enable != 0 && enable != RIANN_PROFILE_ALL && enable != RIANN_PROFILE_DENSE)
        return fail(RIANN_E_INVALID, "profiling level must be 0, RIANN_PROFILE_ALL or RIANN_PROFILE_DENSE");
    if (enable != 0) {
        // fresh totals; events still pending belong to the old ones
        DeviceGuard g(h->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "device sync");
        std::lock_guard<std::mutex> lk(h->pmu);
        for (auto &p : h->pending) {
            h->evpool.push_back(p.a);
            h->evpool.push_back(p.b);
        }
        h->pending.clear();
        for (int k = 0; k < RIANN_K_COUNT; ++k) {
            h->prof_launches[k] = 0;
            h->prof_ms[k] = 0.0;
        }
    }
    h->profiling.store(enable);
    return RIANN_OK;
}

riann_status_t riann_get_profile(riann_index_t h, riann_profile_t *out) {
    if (!h || !out) return fail(RIANN_E_INVALID, "NULL argument");
    DeviceGuard g(h->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device sync");
    std::lock_guard<std::mutex> lk(h->pmu);
    for (auto &p : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            h->prof_ms[p.kind] += ms;
            h->prof_launches[p.kind] += 1;
        }
        h->evpool.push_back(p.a);
        h->evpool.push_back(p.b);
    }
    h->pending.clear();
    for (int k = 0; k < RIANN_K_COUNT; ++k) {
        out->launches[k] = h->prof_launches[k];
        out->ms[k] = h->prof_ms[k];
    }
    return RIANN_OK;
}

riann_status_t riann_build_paper_tables(riann_index_t h, void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    std::lock_guard<std::mutex> lk(h->paper_mu);     // one build per index
    if (h->paper_mem) return RIANN_OK;
    const int64_t n = h->n;
    const int D = h->D;
    if (n > kMaxPaperN) return fail(RIANN_E_UNSUPPORTED, "the paper's tables need n <= 32768");
    const size_t nn = (size_t)n * (size_t)n;
    std::vector<uint32_t> dm, tv;
    std::vector<int32_t> tp;
    try {
        dm.resize(nn);
        tv.resize(nn);
        tp.resize(nn);
    } catch (const std::bad_alloc &) {
        return fail(RIANN_E_NOMEM, "host memory for the n x n tables");
    }
    // pairwise SSD rows, each sorted by (value, index); rows split over threads
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        std::vector<uint64_t> pr((size_t)n);
        for (int64_t i; (i = next.fetch_add(1)) < n;) {
            const uint8_t *ri = &h->ref[(size_t)i * D];
            for (int64_t j = 0; j < n; ++j) {
                const uint8_t *rj = &h->ref[(size_t)j * D];
                uint32_t s = 0;
                for (int k = 0; k < D; ++k) {
                    const int d = (int)ri[k] - (int)rj[k];
                    s += (uint32_t)(d * d);
                }
                dm[(size_t)i * n + j] = s;
                pr[(size_t)j] = ((uint64_t)s << 32) | (uint64_t)j;
            }
            std::sort(pr.begin(), pr.end());
            for (int64_t j = 0; j < n; ++j) {
                tv[(size_t)i * n + j] = (uint32_t)(pr[(size_t)j] >> 32);
                tp[(size_t)i * n + j] = (int32_t)(pr[(size_t)j] & 0xFFFFFFFFu);
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned k = 0; k < nt; ++k) th.emplace_back(work);
    for (auto &x : th) x.join();
    DeviceGuard g(h->device);
    void *mem = nullptr;
    if (hipMalloc(&mem, nn * 12) != hipSuccess)
        return fail(RIANN_E_NOMEM, "hipMalloc of the n x n tables failed");
    hipStream_t st = (hipStream_t)hip_stream;
    char *b = (char *)mem;
    hipError_t e = hipMemcpyAsync(b, dm.data(), nn * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b + nn * 4, tv.data(), nn * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b + nn * 8, tp.data(), nn * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "upload of the n x n tables");
    }
    h->paper_mem = mem;
    return RIANN_OK;
}

riann_status_t riann_match_paper(riann_index_t h, const uint8_t *frame_dev, int32_t H, int32_t W,
                                 int64_t pitch, const int32_t *prev_dev, int32_t *out_dev,
                                 uint32_t *ssd_dev, int32_t *iters_dev, int32_t L, uint64_t seed,
                                 uint64_t t, void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    const void *pmem;
    {
        std::lock_guard<std::mutex> lk(h->paper_mu);
        pmem = h->paper_mem;
    }
    if (!pmem) return fail(RIANN_E_INVALID, "call riann_build_paper_tables first");
    if (L < 1) return fail(RIANN_E_INVALID, "L must be >= 1");
    FrameBatch fb;
    fb.n = 1;
    riann_status_t s = frame_desc(h, frame_dev, H, W, pitch, prev_dev, out_dev, ssd_dev,
                                  RIANN_MODE_RING, &fb.f[0]);
    if (s != RIANN_OK) return s;
    const int64_t Q = (int64_t)fb.f[0].Hq * fb.f[0].Wq;
    if (iters_dev && (overlap(iters_dev, (size_t)Q * 4, out_dev, (size_t)Q * 4) ||
                      overlap(iters_dev, (size_t)Q * 4, ssd_dev, (size_t)Q * 4)))
        return fail(RIANN_E_INVALID, "iters overlaps an output");
    DeviceGuard g(h->device);
    hipStream_t st = (hipStream_t)hip_stream;
    FrameDesc &fd = fb.f[0];
    fd.qbase = 0;
    fd.tbase = 0;
    fb.Q = Q;
    fb.ntiles = ((fd.Wq + kExtTX - 1) / kExtTX) * ((fd.Hq + kExtTY - 1) / kExtTY);
    fb.all_full = 0;
    fb.knn = 1;
    fb.dense_masked = 0;
    Work w;
    s = get_work(h, st, Q, &w);
    if (s != RIANN_OK) return s;
    hipError_t e = launch_extract(h->dix, fb, w, -1, nullptr, st);   // no ring phase: no routing
    if (e != hipSuccess) return hip_fail(e, "k_extract launch");
    const size_t nn = (size_t)h->n * (size_t)h->n;
    const char *b = (const char *)pmem;
    PaperArgs pa{(const uint32_t *)b, (const uint32_t *)(b + nn * 4), (const int32_t *)(b + nn * 8),
                 L, 0, seed, t, iters_dev};
    e = launch_paper(h->dix, fb, w, pa, st);
    if (e != hipSuccess) return hip_fail(e, "k_paper launch");
    h->frames.fetch_add(1);
    return RIANN_OK;
}

riann_status_t riann_stack_frames(const uint8_t *const *frames, int32_t T, int32_t H, int32_t W,
                                  int32_t C, int64_t pitch, uint8_t *out, void *hip_stream) {
    if (!frames || !out) return fail(RIANN_E_INVALID, "frames and out are required");
    if (T < 1 || T > kMaxStack) return fail(RIANN_E_INVALID, "T must be in [1, 16]");
    if (H < 1 || W < 1 || C < 1) return fail(RIANN_E_INVALID, "H, W and C must be >= 1");
    if (pitch < (int64_t)W * C) return fail(RIANN_E_INVALID, "pitch smaller than a row");
    StackArgs sa{};
    const size_t nout = (size_t)H * W * T * C, nin = (size_t)(H - 1) * pitch + (size_t)W * C;
    for (int t = 0; t < T; ++t) {
        if (!frames[t]) return fail(RIANN_E_INVALID, "NULL frame pointer");
        if (overlap(out, nout, frames[t], nin)) return fail(RIANN_E_INVALID, "out overlaps a frame");
        sa.f[t] = frames[t];
    }
    sa.T = T; sa.H = H; sa.W = W; sa.C = C; sa.pitch = pitch; sa.out = out;
    hipError_t e = launch_stack(sa, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "k_stack launch");
    return RIANN_OK;
}

riann_status_t riann_reconstruct(riann_index_t h, const int32_t *field, int32_t H, int32_t W,
                                 const uint8_t *app, int32_t app_channels, float *out,
                                 const uint8_t *gt, int64_t gt_pitch, double *err,
                                 void *hip_stream) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    if (!field || !out) return fail(RIANN_E_INVALID, "field and out are required");
    const int p = h->prm.patch, s = h->prm.stride;
    if (H < p || W < p) return fail(RIANN_E_INVALID, "frame smaller than one patch");
    if (app_channels < 1 || app_channels > 4)
        return fail(RIANN_E_INVALID, "app_channels must be in [1, 4]");
    if (!app && app_channels != h->prm.channels)
        return fail(RIANN_E_INVALID, "without app, app_channels must equal the index's channels");
    if (err && !gt) return fail(RIANN_E_INVALID, "err needs gt");
    if (gt && gt_pitch < (int64_t)W * app_channels)
        return fail(RIANN_E_INVALID, "gt_pitch smaller than a row");
    const int hq = (H - p) / s + 1, wq = (W - p) / s + 1;
    const size_t nout = (size_t)H * W * app_channels * sizeof(float);
    if (overlap(out, nout, field, (size_t)hq * wq * 4) ||
        (app && overlap(out, nout, app, (size_t)h->n * p * p * app_channels)) ||
        (gt && overlap(out, nout, gt, (size_t)(H - 1) * gt_pitch + (size_t)W * app_channels)))
        return fail(RIANN_E_INVALID, "out overlaps an input");
    hipStream_t st = (hipStream_t)hip_stream;
    DeviceGuard g(h->device);
    ReconArgs ra{field, hq, wq, H, W, app_channels, app, out, gt, gt_pitch, nullptr};
    if (err) {
        const int64_t nb = recon_blocks(H, W);
        std::lock_guard<std::mutex> lk(h->mu);
        auto &sc = h->recon_scratch[st];
        if (sc.second < nb) {
            if (sc.first) {
                hipError_t e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(e, "stream sync");
                (void)hipFree(sc.first);
                sc = {nullptr, 0};
            }
            void *pp = nullptr;
            if (hipMalloc(&pp, (size_t)nb * 3 * sizeof(double)) != hipSuccess)
                return fail(RIANN_E_NOMEM, "hipMalloc of reconstruction scratch failed");
            sc = {(double *)pp, nb};
        }
        ra.partials = sc.first;
    }
    hipError_t e = launch_recon(h->dix, ra, err, st);
    if (e != hipSuccess) return hip_fail(e, "k_recon launch");
    return RIANN_OK;
}

riann_status_t riann_destroy(riann_index_t h) {
    if (!h) return fail(RIANN_E_INVALID, "index is NULL");
    free_index(h);
    return RIANN_OK;
}

}  // extern "C"
