// Pixel matching cost M(v, label) of the restricted cost volume (Section 3.3,
// eq. E): truncated colour term plus truncated gradient term.  Shared by the
// cost-volume kernel and the fused up pass, so both produce the same floats.
#pragma once

#include "common.hpp"

namespace hdp {

struct CostParams {
    float a_c, tau_c, a_g, tau_g;
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
    return outside ? sat : m;
}

__device__ __forceinline__ float match_cost(float4 L, const float4 *__restrict__ right, int v,
                                            int x, int label, const CostParams &c) {
    return match_cost_px(L, right[match_src(v, x, label)], x - label < 0, c);
}

}  // namespace hdp
