// Graph pyramid (Section 2.1) and pixel interval prediction (Section 3.1).
#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

// Layer 0: uint8 RGB -> (R, G, B, gx) with gx = sum(x+1) - sum(x-1) (replicated
// border); every value is an exact small integer in FP32.
__global__ void k_level0(const uint8_t *__restrict__ rgb, LevelGeom g, float4 *__restrict__ out) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    PixelPos p = pixel_pos(g, (int)v);
    const uint8_t *c = rgb + 3 * v;
    int xr = p.x + 1 < p.W ? 1 : 0;
    int xl = p.x > 0 ? -1 : 0;
    const uint8_t *cr = rgb + 3 * (v + xr);
    const uint8_t *cl = rgb + 3 * (v + xl);
    float sr = (float)((int)cr[0] + cr[1] + cr[2]);
    float sl = (float)((int)cl[0] + cl[1] + cl[2]);
    out[v] = make_float4((float)c[0], (float)c[1], (float)c[2], sr - sl);
}

// Layer l+1 from layer l: mean over the children of the S x S square that lie
// inside the image (S = 2: 1, 2 or 4 children, so the mean is exact).
__global__ void k_downsample(const float4 *__restrict__ in, LevelGeom gi, float4 *__restrict__ out,
                             LevelGeom go, int S) {
    int64_t V = gtid();
    if (V >= go.off[go.n_pairs]) return;
    PixelPos P = pixel_pos(go, (int)V);
    int Wi = gi.W[P.pair], Hi = gi.H[P.pair], bi = gi.off[P.pair];
    float r = 0.f, gg = 0.f, b = 0.f;
    int cnt = 0;
    for (int dy = 0; dy < S; ++dy) {
        int y = S * P.y + dy;
        if (y >= Hi) break;
        for (int dx = 0; dx < S; ++dx) {
            int x = S * P.x + dx;
            if (x >= Wi) break;
            float4 c = in[bi + y * Wi + x];
            r += c.x; gg += c.y; b += c.z;
            ++cnt;
        }
    }
    float inv = 1.0f / (float)cnt;  // 1, 1/2, 1/4: exact
    out[V] = make_float4(r * inv, gg * inv, b * inv, 0.f);
}

// Fill the gx channel of a layer from the channel sums of its row neighbours.
__global__ void k_gradient(float4 *__restrict__ img, LevelGeom g) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    PixelPos p = pixel_pos(g, (int)v);
    int xr = p.x + 1 < p.W ? 1 : 0;
    int xl = p.x > 0 ? -1 : 0;
    float4 a = img[v + xr];
    float4 b = img[v + xl];
    float sr = (a.x + a.y) + a.z;
    float sl = (b.x + b.y) + b.z;
    reinterpret_cast<float *>(img)[4 * v + 3] = sr - sl;
}

// PixelIntv = [S*i - w, S*i + S - 1 + w] clipped to [0, dmax_l], i = label of
// the covering node one layer up.
__global__ void k_predict_range(const int32_t *__restrict__ disp_up, LevelGeom gu, LevelGeom gl,
                                int S, int window, int32_t *__restrict__ lo,
                                int32_t *__restrict__ hi) {
    int64_t v = gtid();
    if (v >= gl.off[gl.n_pairs]) return;
    PixelPos p = pixel_pos(gl, (int)v);
    int i = disp_up[gu.off[p.pair] + (p.y / S) * gu.W[p.pair] + p.x / S];
    int a = S * i - window, b = S * i + S - 1 + window;
    int dl = gl.dmax[p.pair];
    lo[v] = a < 0 ? 0 : a;
    hi[v] = b > dl ? dl : b;
}

void launch_pyramid(const uint8_t *rgb, const LevelGeom *geoms, int L, int S, float *levels,
                    hipStream_t st) {
    float4 *cur = reinterpret_cast<float4 *>(levels);
    int64_t n0 = geoms[0].off[geoms[0].n_pairs];
    k_level0<<<grid_for(n0), kBlock, 0, st>>>(rgb, geoms[0], cur);
    for (int l = 0; l < L; ++l) {
        int64_t ni = geoms[l].off[geoms[l].n_pairs];
        int64_t no = geoms[l + 1].off[geoms[l + 1].n_pairs];
        float4 *nxt = cur + ni;
        k_downsample<<<grid_for(no), kBlock, 0, st>>>(cur, geoms[l], nxt, geoms[l + 1], S);
        k_gradient<<<grid_for(no), kBlock, 0, st>>>(nxt, geoms[l + 1]);
        cur = nxt;
    }
}

void launch_predict_range(const int32_t *disp_up, const LevelGeom &gu, const LevelGeom &gl, int S,
                          int window, int32_t *lo, int32_t *hi, hipStream_t st) {
    int64_t n = gl.off[gl.n_pairs];
    k_predict_range<<<grid_for(n), kBlock, 0, st>>>(disp_up, gu, gl, S, window, lo, hi);
}

}  // namespace hdp
