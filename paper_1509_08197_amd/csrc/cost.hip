// Restricted matching cost E (Section 3.3, eq. E) and winner-takes-all.
#include "common.hpp"
#include "kernels.hpp"
#include "matchcost.hpp"

namespace hdp {

// One thread per CPT consecutive columns of a row (vector stores); a
// workgroup covers kBlock / (width / CPT) whole rows.  node == NULL: rows are
// pixels and the interval is [0, dmax of the pair].
template <int CPT>
__global__ void __launch_bounds__(kBlock) k_cost_volume(
    const float4 *__restrict__ left, const float4 *__restrict__ right, LevelGeom g,
    const int32_t *__restrict__ node, const int32_t *__restrict__ lo,
    const int32_t *__restrict__ hi, int width, CostParams cp, float *__restrict__ cost) {
    const int lpr = width / CPT;
    const int rows_per_block = kBlock / lpr;
    const int gi = threadIdx.x / lpr;
    if (gi >= rows_per_block) return;
    const int j0 = (threadIdx.x - gi * lpr) * CPT;
    const int64_t r = (int64_t)blockIdx.x * rows_per_block + gi;
    if (r >= g.off[g.n_pairs]) return;
    const int v = node ? node[r] : (int)r;
    const PixelPos p = pixel_pos(g, v);
    const int a = node ? lo[v] : 0;
    const int b = node ? hi[v] : g.dmax[p.pair];
    const float4 L = left[v];
    float4 R[CPT];  // every right pixel is read before any is used
#pragma unroll
    for (int c = 0; c < CPT; ++c) R[c] = right[match_src(v, p.x, a + j0 + c)];
    float out[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        int label = a + j0 + c;
        out[c] = label <= b ? match_cost_px(L, R[c], p.x - label < 0, cp) : 0.f;
    }
    float *dst = cost + r * width + j0;
    if (CPT == 4)
        *reinterpret_cast<float4 *>(dst) = make_float4(out[0], out[1], out[2], out[3]);
    else if (CPT == 2)
        *reinterpret_cast<float2 *>(dst) = make_float2(out[0], out[1]);
    else
        dst[0] = out[0];
}

// Winner-takes-all: LPR consecutive lanes take one row (lane j reads columns
// j, j + LPR, ..., so the row is read by consecutive lanes); each lane keeps
// its least value and column (first of equal values), then a butterfly over
// the row's lanes keeps the least value, the lower column on ties.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_wta(LevelGeom g, const int32_t *__restrict__ node,
                                                const int32_t *__restrict__ lo,
                                                const int32_t *__restrict__ hi, int width,
                                                const float *__restrict__ agg,
                                                int32_t *__restrict__ disp, int64_t n) {
    const int64_t r = gtid() / LPR;
    const int j = (int)(threadIdx.x & (LPR - 1));
    float best = __builtin_inff();
    int bj = 0x7fffffff;
    int v = 0, a = 0;
    if (r < n) {
        v = node ? node[r] : (int)r;
        a = node ? lo[v] : 0;
        const int b = node ? hi[v] : g.dmax[pair_of(g, v)];
        const int nl = b - a + 1 < width ? b - a + 1 : width;
        const float *row = agg + r * width;
        for (int x = j; x < nl; x += LPR) {
            const float y = row[x];
            if (y < best) {
                best = y;
                bj = x;
            }
        }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (ob < best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
    }
    if (r < n && j == 0) disp[v] = a + (bj == 0x7fffffff ? 0 : bj);
}

void launch_cost_volume(const float *left, const float *right, const LevelGeom &g,
                        const int32_t *node, const int32_t *lo, const int32_t *hi, int width,
                        const hdp_cost_params &p, float *cost, hipStream_t st) {
    int64_t n = g.off[g.n_pairs];
    CostParams cp{p.a_c, p.tau_c, p.a_g, p.tau_g, p.border};
    const float4 *L = reinterpret_cast<const float4 *>(left);
    const float4 *R = reinterpret_cast<const float4 *>(right);
    int cpt = (width % 4 == 0 && width / 4 <= kBlock) ? 4 : (width % 2 == 0 ? 2 : 1);
    int lpr = width / cpt;
    int rpb = kBlock / lpr;
    unsigned blocks = (unsigned)((n + rpb - 1) / rpb);
    timer_before(HDP_TIMER_COST, st);
    if (cpt == 4)
        k_cost_volume<4><<<blocks, kBlock, 0, st>>>(L, R, g, node, lo, hi, width, cp, cost);
    else if (cpt == 2)
        k_cost_volume<2><<<blocks, kBlock, 0, st>>>(L, R, g, node, lo, hi, width, cp, cost);
    else
        k_cost_volume<1><<<blocks, kBlock, 0, st>>>(L, R, g, node, lo, hi, width, cp, cost);
    timer_after(HDP_TIMER_COST, st);
}

void launch_wta(const LevelGeom &g, const int32_t *node, const int32_t *lo, const int32_t *hi,
                int width, const float *agg, int32_t *disp, hipStream_t st) {
    const int64_t n = g.off[g.n_pairs];
    const int lpr = width <= 16 ? 4 : width <= 32 ? 8 : width <= 64 ? 16 : width <= 128 ? 32 : 64;
#define HDP_WTA(L) k_wta<L><<<grid_for(n * L), kBlock, 0, st>>>(g, node, lo, hi, width, agg, disp, n)
    if (lpr == 4) HDP_WTA(4);
    else if (lpr == 8) HDP_WTA(8);
    else if (lpr == 16) HDP_WTA(16);
    else if (lpr == 32) HDP_WTA(32);
    else HDP_WTA(64);
#undef HDP_WTA
}

}  // namespace hdp
