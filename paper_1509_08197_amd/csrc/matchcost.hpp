// Pixel matching cost M(v, label) of the restricted cost volume (Section 3.3,
// eq. E): truncated colour term plus truncated gradient term.  Shared by the
// cost-volume kernel and the fused up pass, so both produce the same floats.
#pragma once

#include "common.hpp"

namespace hdp {

struct CostParams {
    float a_c, tau_c, a_g, tau_g;
};

// Colour term from the channel differences, gradient term from the difference
// of the gx numerators (gray gradient = gx / 6).  A label that reaches past the
// left image border costs both truncations.
__device__ __forceinline__ float match_cost(float4 L, const float4 *__restrict__ right, int v,
                                            int x, int label, const CostParams &c) {
    // no contraction into FMAs: every kernel that inlines this computes the same floats
#pragma clang fp contract(off)
    if (x - label < 0) return c.a_c * c.tau_c + c.a_g * c.tau_g;
    float4 R = right[v - label];
    float col = (fabsf(L.x - R.x) + fabsf(L.y - R.y) + fabsf(L.z - R.z)) / 3.0f;
    float gd = fabsf(L.w - R.w) / 6.0f;
    return c.a_c * fminf(col, c.tau_c) + c.a_g * fminf(gd, c.tau_g);
}

}  // namespace hdp
