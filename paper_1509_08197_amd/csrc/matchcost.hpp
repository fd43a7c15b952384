// Pixel matching cost M(v, label) of the restricted cost volume (Section 3.3,
// eq. E): truncated colour term plus truncated gradient term.  Shared by the
// cost-volume kernel and the fused up pass, so both produce the same floats.
#pragma once

#include "common.hpp"

namespace hdp {

struct CostParams {
    float a_c, tau_c, a_g, tau_g;
    int border;  // 0: a match past the left border costs both truncations; 1: row's first pixel
};

// Right-image pixel that label `label` of pixel v (column x) is compared with.
// A label reaching past the left border is clamped to the row's first pixel:
// the read stays inside the image and its value is not used (see below), so
// callers can issue the load before they know whether it is needed.
__device__ __forceinline__ int match_src(int v, int x, int label) {
    return v - (label < x ? label : x);
}

// Cost from the two pixels: colour term from the channel differences,
// gradient term from the difference of the gx numerators (gray gradient =
// gx / 6).  A label that reaches past the left image border (outside) costs
// both truncations.  The means are taken by multiplying with the rounded
// reciprocals 1/3 and 1/6 (within an ulp of the quotients, and far cheaper
// than a correctly rounded division).
__device__ __forceinline__ float match_cost_px(float4 L, float4 R, bool outside,
                                               const CostParams &c) {
    // no contraction into FMAs: every kernel that inlines this computes the same floats
#pragma clang fp contract(off)
    const float col = (fabsf(L.x - R.x) + fabsf(L.y - R.y) + fabsf(L.z - R.z)) * (1.0f / 3.0f);
    const float gd = fabsf(L.w - R.w) * (1.0f / 6.0f);
    const float m = c.a_c * fminf(col, c.tau_c) + c.a_g * fminf(gd, c.tau_g);
    const float sat = c.a_c * c.tau_c + c.a_g * c.tau_g;
    return outside && c.border == 0 ? sat : m;
}

// Right-image pixel in 8 bytes for the fused up pass: R, G and B times 4^l
// in 14 bits each and the gradient numerator times 4^l in 22 bits (two's
// complement), l the pyramid layer.  Exact for the pixels of a pyramid of 2x2
// means at layers 0..3 (multiples of 4^-l, channels at most 255, |gx| at most
// 765): unpacking gives back the same floats.  Any other pixel is stored as
// all ones (a red field of 16383, which no packed pixel has) and is read as
// its FP32 value instead.
__device__ __forceinline__ uint2 pack_right(float4 p, float scale) {
    const float r = p.x * scale, g = p.y * scale, b = p.z * scale, x = p.w * scale;
    const bool ok = r >= 0.f && r < 16383.f && r == rintf(r) && g >= 0.f && g < 16383.f &&
                    g == rintf(g) && b >= 0.f && b < 16383.f && b == rintf(b) &&
                    fabsf(x) < 2097152.f && x == rintf(x);
    if (!ok) return make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
    const uint32_t R = (uint32_t)r, G = (uint32_t)g, B = (uint32_t)b;
    const uint32_t X = (uint32_t)(int32_t)x & 0x3FFFFFu;
    return make_uint2(R | (G << 14) | (B << 28), (B >> 4) | (X << 10));
}
__device__ __forceinline__ bool packed_fallback(uint2 q) { return (q.x & 0x3FFFu) == 0x3FFFu; }
// inv = 4^-l
__device__ __forceinline__ float4 unpack_right(uint2 q, float inv) {
    const float R = (float)(q.x & 0x3FFFu), G = (float)((q.x >> 14) & 0x3FFFu);
    const float B = (float)((q.x >> 28) | ((q.y & 0x3FFu) << 4));
    const float X = (float)((int32_t)q.y >> 10);
    return make_float4(R * inv, G * inv, B * inv, X * inv);
}

__device__ __forceinline__ float match_cost(float4 L, const float4 *__restrict__ right, int v,
                                            int x, int label, const CostParams &c) {
    return match_cost_px(L, right[match_src(v, x, label)], x - label < 0, c);
}

}  // namespace hdp
