// Left-right consistency check, sampled label prior and the cost of the
// tree-based refinement (Sections 3.1 and 3.3).
//
// The right view's labels come from the method run on the horizontally
// mirrored pair with the right image as reference (hdp_mirror gives the
// inputs); a left pixel (x, y) with label d is stable when x - d is inside the
// image and the right view's label there is within tol of d.  The prior
// P(D_l) counts the labels of the stable centres of square x square blocks.
// The refinement cost of a stable pixel is |x - D(p)| at label x (0 for an
// unstable one); aggregated over the layer's forest and reduced by the
// winner-takes-all it pulls every pixel towards the stable labels near it on
// the tree.  All of it is integer work except the cost, which is an exact
// small integer in FP32.
#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

// out(x, y) = in(W - 1 - x, y), interleaved RGB bytes.
__global__ void k_mirror(const uint8_t *__restrict__ in, LevelGeom g, uint8_t *__restrict__ out) {
    const int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    const PixelPos p = pixel_pos(g, (int)v);
    const int64_t src = p.base + (int64_t)p.y * p.W + (p.W - 1 - p.x);
    const uint8_t r = in[3 * src], gg = in[3 * src + 1], b = in[3 * src + 2];
    out[3 * v] = r;
    out[3 * v + 1] = gg;
    out[3 * v + 2] = b;
}

__global__ void k_lr_check(const int32_t *__restrict__ dl, const int32_t *__restrict__ dr,
                           int right_mirrored, LevelGeom g, int tol,
                           uint8_t *__restrict__ stable) {
    const int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    const PixelPos p = pixel_pos(g, (int)v);
    const int d = dl[v], xr = p.x - d;
    uint8_t ok = 0;
    if (xr >= 0 && xr < p.W) {
        const int xc = right_mirrored ? p.W - 1 - xr : xr;
        const int e = dr[p.base + (int64_t)p.y * p.W + xc];
        ok = (d - e <= tol) && (e - d <= tol);
    }
    stable[v] = ok;
}

__global__ void k_zero_f64(double *p, int64_t n) {
    for (int64_t i = gtid(); i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

// One thread per block centre (square/2 + k*square in both directions, inside
// the image) of every pair; ct = first centre of each pair (host-computed).
__global__ void k_sample_prior(const int32_t *__restrict__ disp, const uint8_t *__restrict__ stable,
                               LevelGeom g, int square, CentreTable ct, double *__restrict__ prior,
                               int prior_stride) {
    const int64_t t = gtid();
    if (t >= ct.off[g.n_pairs]) return;
    int pair = 0;
    while (pair + 1 < g.n_pairs && ct.off[pair + 1] <= t) ++pair;
    const int k = (int)(t - ct.off[pair]);
    const int cy = k / ct.nx[pair], cx = k - cy * ct.nx[pair];
    const int64_t v = g.off[pair] + (int64_t)(square / 2 + cy * square) * g.W[pair] +
                      (square / 2 + cx * square);
    const int d = disp[v];
    if (stable[v] && d >= 0 && d <= g.dmax[pair])
        atomicAdd(&prior[(int64_t)pair * prior_stride + d], 1.0);  // integer counts: exact
}

// Refinement cost in the forest's volume layout: row r (pixel v = node[r])
// holds labels lo(v) + c, c = 0 .. width-1; padding columns past hi(v) are 0.
__global__ void k_refine_cost(const int32_t *__restrict__ disp, const uint8_t *__restrict__ stable,
                              const int32_t *__restrict__ node, const int32_t *__restrict__ lo,
                              const int32_t *__restrict__ hi, int64_t n, int width,
                              float *__restrict__ cost) {
    const int64_t t = gtid();
    if (t >= n * width) return;
    const int64_t r = t / width;
    const int c = (int)(t - r * width);
    const int v = node[r];
    const int x = lo[v] + c;
    const int d = disp[v];
    const uint8_t s = stable[v];
    const int h = hi[v];
    float out = 0.f;
    if (x <= h && s) out = (float)(x > d ? x - d : d - x);
    cost[t] = out;
}

void launch_mirror(const uint8_t *in, const LevelGeom &g, uint8_t *out, hipStream_t st) {
    const int64_t n = g.off[g.n_pairs];
    k_mirror<<<grid_for(n), kBlock, 0, st>>>(in, g, out);
}

void launch_lr_check(const int32_t *dl, const int32_t *dr, int right_mirrored, const LevelGeom &g,
                     int tol, uint8_t *stable, hipStream_t st) {
    const int64_t n = g.off[g.n_pairs];
    k_lr_check<<<grid_for(n), kBlock, 0, st>>>(dl, dr, right_mirrored, g, tol, stable);
}

void launch_sample_prior(const int32_t *disp, const uint8_t *stable, const LevelGeom &g,
                         int square, double *prior, int prior_stride, hipStream_t st) {
    CentreTable ct{};
    int64_t tot = 0;
    for (int p = 0; p < g.n_pairs; ++p) {
        const int nx = g.W[p] > square / 2 ? (g.W[p] - square / 2 + square - 1) / square : 0;
        const int ny = g.H[p] > square / 2 ? (g.H[p] - square / 2 + square - 1) / square : 0;
        ct.off[p] = tot;
        ct.nx[p] = nx > 0 ? nx : 1;
        tot += (int64_t)nx * ny;
    }
    ct.off[g.n_pairs] = tot;
    const int64_t words = (int64_t)g.n_pairs * prior_stride;
    k_zero_f64<<<grid_for(words), kBlock, 0, st>>>(prior, words);
    if (tot > 0)
        k_sample_prior<<<grid_for(tot), kBlock, 0, st>>>(disp, stable, g, square, ct, prior,
                                                         prior_stride);
}

void launch_refine_cost(const int32_t *disp, const uint8_t *stable, const hdp_forest &f,
                        int width, float *cost, hipStream_t st) {
    k_refine_cost<<<grid_for(f.n * width), kBlock, 0, st>>>(disp, stable, f.node, f.lo, f.hi, f.n,
                                                            width, cost);
}

}  // namespace hdp
