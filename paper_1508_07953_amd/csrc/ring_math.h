// ring_math.h -- integer distance and ring-size arithmetic shared by the ring
// phase (k_ring.hip) and the extraction kernel that routes queries on the
// same ring-size bounds (k_extract.hip).
#pragma once
#include "riann_internal.h"

namespace riann {

// The hardware square root (v_sqrt_f32, about 1 ulp).  Its arguments here are
// SSDs and products of two SSDs as fp32, zero or at least 1 (no denormal
// inputs).  Every bound below widens its estimate by a relative 2^-18, 32 ulps,
// far above this error, so the correctly rounded library sqrtf (a dozen more
// instructions) is not needed.
__device__ __forceinline__ float sqrt_est(float x) { return __builtin_amdgcn_sqrtf(x); }

// <a, v> over DP bytes: a in registers, v a 16-byte aligned reference row.
template <int DP>
__device__ __forceinline__ int dot_row(const uint32_t (&a)[DP / 4], const int8_t *__restrict__ v) {
    const uint4 *v4 = reinterpret_cast<const uint4 *>(v);
    int acc = 0;
#pragma unroll
    for (int i = 0; i < DP / 16; ++i) {
        uint4 r = v4[i];
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 0], (int)r.x, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 1], (int)r.y, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 2], (int)r.z, acc, false);
        acc = __builtin_amdgcn_sdot4((int)a[4 * i + 3], (int)r.w, acc, false);
    }
    return acc;
}

// An inner and an outer approximation of key k's ring: s = floor(sqrt(4bc))
// lies in [s_in, s_out] for the fp32 estimate widened by a relative 2^-18
// (far above the rounding of the product, the square root and the scaling)
// and one unit, so [lo_in, hi_in] lies inside the exact ring and
// [lo_out, hi_out] contains it.
__device__ __forceinline__ void ring_approx(uint32_t b, uint32_t c, uint32_t &lo_in,
                                            uint32_t &hi_in, uint32_t &lo_out, uint32_t &hi_out) {
    const float sf = 2.0f * sqrt_est((float)b * (float)c);
    const float si = floorf(sf * (1.0f - 0x1p-18f)) - 1.0f;
    const float so = ceilf(sf * (1.0f + 0x1p-18f)) + 1.0f;
    // b, c are SSDs (< 2^24): s <= 2^25 + 2 and every end below 2^27, so the
    // arithmetic stays in 32 bits
    const uint32_t s_in = si > 0.0f ? (uint32_t)si : 0u, s_out = (uint32_t)so;
    const uint32_t bc = b + c;
    lo_in = b <= c ? 0u : bc - min(s_in, bc);
    hi_in = bc + s_in;
    lo_out = b <= c ? 0u : bc - min(s_out, bc);
    hi_out = bc + s_out;
}

// Bounds on the number of key-list entries inside the exact ring from the
// key's bucket counts (row {vmin, shift, cdf[0..B]}): the whole buckets
// inside [lo_in, hi_in] give lb, the buckets meeting [lo_out, hi_out] give ub.
__device__ __forceinline__ void ring_size_bounds(const uint32_t *row, int B, uint32_t lo_in,
                                                 uint32_t hi_in, uint32_t lo_out, uint32_t hi_out,
                                                 uint32_t &lb, uint32_t &ub) {
    // ring ends are below 2^27 and the bucket shift is at most 24 (a key's
    // distances span less than 2^24), so 32-bit arithmetic is exact
    const uint32_t vmin = row[0], sh = row[1];
    const uint32_t wm = (1u << sh) - 1u;
    // entries below vmin + d: d from the interval's ends
    auto below = [&](uint32_t v, bool incl) -> uint32_t {
        return v >= vmin ? v - vmin + (incl ? 1u : 0u) : 0u;
    };
    const uint32_t dli = below(lo_in, false), dhi = below(hi_in, true);
    const uint32_t dlo = below(lo_out, false), dho = below(hi_out, true);
    const uint32_t ub_ = (uint32_t)B;
    const uint32_t jl_in = min(ub_, (dli + wm) >> sh);
    const uint32_t jh_in = min(ub_, dhi >> sh);
    const uint32_t jl_out = min(ub_, dlo >> sh);
    const uint32_t jh_out = min(ub_, (dho + wm) >> sh);
    lb = jh_in > jl_in ? row[2 + jh_in] - row[2 + jl_in] : 0u;
    ub = jh_out > jl_out ? row[2 + jh_out] - row[2 + jl_out] : 0u;
}

// The lower bound alone of ring_size_bounds: entries of key k's sorted list
// certainly inside the exact ring of (b, c), from the key's bucket counts.
__device__ __forceinline__ uint32_t ring_lower_bound(const uint32_t *row, int B, uint32_t b,
                                                     uint32_t c) {
    uint32_t li, hi_, lo_, ho, lb, ub;
    ring_approx(b, c, li, hi_, lo_, ho);
    ring_size_bounds(row, B, li, hi_, lo_, ho, lb, ub);
    return lb;
}

// Entries of a key's sorted list certainly inside the ring of (b, c), from
// its routing row (square-root space): with sb ~ sqrt(b), sc ~ sqrt(c) (fp32),
// every entry a with sqrt(a) in [o + jl 2^e, o + jh 2^e) lies in
// [sqrt(b) - sqrt(c), sqrt(b) + sqrt(c)], i.e. in the exact ring, when jl and
// jh are rounded inward from sb -/+ sc by a margin eps far above the fp32
// errors of the square roots, sums and differences ((sb + sc + o) 2^-18 +
// 2^-8 against at most a few units in 2^-22 relative).  The scaling by 2^-e
// is exact.
__device__ __forceinline__ uint32_t route_lower_bound(const uint32_t *row, float sb, float sc) {
    const float o = __uint_as_float(row[0]), inv = __uint_as_float(row[1]);
    const float eps = (sb + sc + o) * 0x1p-18f + 0x1p-8f;
    const float tl = ((sb - sc) - o + eps) * inv;
    const float th = ((sb + sc) - o - eps) * inv;
    const float B = (float)kRouteBuckets;
    const int jl = (int)fminf(fmaxf(ceilf(tl), 0.0f), B);
    const int jh = (int)fminf(fmaxf(floorf(th), 0.0f), B);
    return jh > jl ? row[2 + jh] - row[2 + jl] : 0u;
}

}  // namespace riann
