// Graph pyramid (Section 2.1) and pixel interval prediction (Section 3.1).
#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

// One launch serves the two views of a pair batch: blockIdx.y selects the
// view (rgb / level buffers of view y).
struct Views {
    const uint8_t *rgb[2];
    float4 *lev[2];  // layer buffers of the current output layer
    const float4 *src[2];  // layer buffers of the input layer (downsampling)
};

// Layer 0: uint8 RGB -> (R, G, B, gx) with gx = sum(x+1) - sum(x-1) (replicated
// border); every value is an exact small integer in FP32.
__global__ void k_level0(Views V, LevelGeom g) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    const uint8_t *rgb = V.rgb[blockIdx.y];
    PixelPos p = pixel_pos(g, (int)v);
    const uint8_t *c = rgb + 3 * v;
    int xr = p.x + 1 < p.W ? 1 : 0;
    int xl = p.x > 0 ? -1 : 0;
    const uint8_t *cr = rgb + 3 * (v + xr);
    const uint8_t *cl = rgb + 3 * (v + xl);
    float sr = (float)((int)cr[0] + cr[1] + cr[2]);
    float sl = (float)((int)cl[0] + cl[1] + cl[2]);
    V.lev[blockIdx.y][v] = make_float4((float)c[0], (float)c[1], (float)c[2], sr - sl);
}

// The same, four pixels per thread, for 4-byte aligned RGB buffers: the bytes
// of pixels v0-1 .. v0+4 come in five aligned 32-bit loads (one per thread
// and 4 bytes instead of six narrow loads per pixel).  Threads whose words
// would reach outside the buffer (the first and the last few) take the
// pixels one by one.
__device__ __forceinline__ uint32_t rgb_sum(const uint32_t *w, int px) {
    // bytes 3 px .. 3 px + 2 of the byte string held by w[-1 ..] (px >= -1)
    int s = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b = 3 * px + c + 4;  // w[-1] holds bytes -4 .. -1
        s += (int)((w[(b >> 2) - 1] >> (8 * (b & 3))) & 255u);
    }
    return (uint32_t)s;
}
__device__ __forceinline__ float4 rgb_px(const uint32_t *w, int px) {
    float f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b = 3 * px + c + 4;
        f[c] = (float)((w[(b >> 2) - 1] >> (8 * (b & 3))) & 255u);
    }
    return make_float4(f[0], f[1], f[2], 0.f);
}

__global__ void __launch_bounds__(kBlock) k_level0_x4(Views V, LevelGeom g) {
    __shared__ float4 stage[4 * kBlock];
    const int64_t t = gtid();
    const int64_t n = g.off[g.n_pairs];
    const int64_t v0 = 4 * t;
    const uint8_t *rgb = V.rgb[blockIdx.y];
    float4 *out = V.lev[blockIdx.y];
    float4 c[4];
    if (v0 >= n) {
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else if (t == 0 || v0 + 8 > n) {  // words outside the buffer: pixel by pixel
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t v = v0 + i < n ? v0 + i : n - 1;
            const PixelPos p = pixel_pos(g, (int)v);
            const uint8_t *cv = rgb + 3 * v;
            const uint8_t *cr = rgb + 3 * (v + (p.x + 1 < p.W ? 1 : 0));
            const uint8_t *cl = rgb + 3 * (v - (p.x > 0 ? 1 : 0));
            const float sr = (float)((int)cr[0] + cr[1] + cr[2]);
            const float sl = (float)((int)cl[0] + cl[1] + cl[2]);
            c[i] = make_float4((float)cv[0], (float)cv[1], (float)cv[2], sr - sl);
        }
    } else {
        // w[0] .. w[4] = words 3t - 1 .. 3t + 3 (bytes 12t - 4 .. 12t + 15)
        const uint32_t *src = reinterpret_cast<const uint32_t *>(rgb) + 3 * t - 1;
        uint32_t w[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) w[k] = src[k];
        const uint32_t *wp = w + 1;  // wp[-1] holds bytes -4 .. -1 of the thread's 12
        float sum[6];                 // channel sums of pixels v0 - 1 .. v0 + 4
#pragma unroll
        for (int k = 0; k < 6; ++k) sum[k] = (float)rgb_sum(wp, k - 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const PixelPos p = pixel_pos(g, (int)(v0 + i));
            const float sr = p.x + 1 < p.W ? sum[i + 2] : sum[i + 1];
            const float sl = p.x > 0 ? sum[i] : sum[i + 1];
            c[i] = rgb_px(wp, i);
            c[i].w = sr - sl;
        }
    }
    // through LDS, so that every store instruction writes consecutive pixels
#pragma unroll
    for (int i = 0; i < 4; ++i) stage[4 * threadIdx.x + i] = c[i];
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * kBlock * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t v = b0 + k * kBlock + threadIdx.x;
        if (v < n) out[v] = stage[k * kBlock + threadIdx.x];
    }
}

// Mean over the children of the S x S square of node (X, Y) that lie inside
// layer l (S = 2: 1, 2 or 4 children, so the mean is exact).
__device__ __forceinline__ float3 square_mean(const float4 *__restrict__ in, int bi, int Wi, int Hi,
                                              int X, int Y, int S) {
    float r = 0.f, gg = 0.f, b = 0.f;
    int cnt = 0;
    for (int dy = 0; dy < S; ++dy) {
        int y = S * Y + dy;
        if (y >= Hi) break;
        for (int dx = 0; dx < S; ++dx) {
            int x = S * X + dx;
            if (x >= Wi) break;
            float4 c = in[bi + y * Wi + x];
            r += c.x; gg += c.y; b += c.z;
            ++cnt;
        }
    }
    float inv = 1.0f / (float)cnt;  // 1, 1/2, 1/4: exact
    return make_float3(r * inv, gg * inv, b * inv);
}

// Layer l+1 from layer l (Section 2.1), with its gx channel from the channel
// sums of the row neighbours' means (replicated border).
__global__ void k_downsample(Views V, LevelGeom gi, LevelGeom go, int S) {
    int64_t Vx = gtid();
    if (Vx >= go.off[go.n_pairs]) return;
    const float4 *in = V.src[blockIdx.y];
    PixelPos P = pixel_pos(go, (int)Vx);
    int Wi = gi.W[P.pair], Hi = gi.H[P.pair], bi = gi.off[P.pair];
    int xr = P.x + 1 < P.W ? P.x + 1 : P.x;
    int xl = P.x > 0 ? P.x - 1 : P.x;
    float3 m, a, b;
    if (S == 2) {
        // the 2 x 2 squares of the node and its row neighbours: all 12 child
        // loads issued at once (clamped), then the means in the order of
        // square_mean (row by row, left to right)
        const int y0 = 2 * P.y, y1 = 2 * P.y + 1 < Hi ? 2 * P.y + 1 : 2 * P.y;
        const bool hy = 2 * P.y + 1 < Hi;
        int cx[6];
        bool hx[3];
        const int nx[3] = {xl, P.x, xr};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cx[2 * k] = 2 * nx[k];
            hx[k] = 2 * nx[k] + 1 < Wi;
            cx[2 * k + 1] = hx[k] ? 2 * nx[k] + 1 : 2 * nx[k];
        }
        float4 c0[6], c1[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            c0[q] = in[bi + y0 * Wi + cx[q]];
            c1[q] = in[bi + y1 * Wi + cx[q]];
        }
        float3 mm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float r = c0[2 * k].x, gg = c0[2 * k].y, bb = c0[2 * k].z;
            int cnt = 1;
            if (hx[k]) { r += c0[2 * k + 1].x; gg += c0[2 * k + 1].y; bb += c0[2 * k + 1].z; ++cnt; }
            if (hy) {
                r += c1[2 * k].x; gg += c1[2 * k].y; bb += c1[2 * k].z; ++cnt;
                if (hx[k]) { r += c1[2 * k + 1].x; gg += c1[2 * k + 1].y; bb += c1[2 * k + 1].z; ++cnt; }
            }
            const float inv = 1.0f / (float)cnt;  // 1, 1/2, 1/4: exact
            mm[k] = make_float3(r * inv, gg * inv, bb * inv);
        }
        b = mm[0];
        m = mm[1];
        a = mm[2];
    } else {
        m = square_mean(in, bi, Wi, Hi, P.x, P.y, S);
        a = xr == P.x ? m : square_mean(in, bi, Wi, Hi, xr, P.y, S);
        b = xl == P.x ? m : square_mean(in, bi, Wi, Hi, xl, P.y, S);
    }
    float sr = (a.x + a.y) + a.z;
    float sl = (b.x + b.y) + b.z;
    V.lev[blockIdx.y][Vx] = make_float4(m.x, m.y, m.z, sr - sl);
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

void launch_pyramid(const uint8_t *const *rgb, int views, const LevelGeom *geoms, int L, int S,
                    float *const *levels, hipStream_t st) {
    Views V{};
    for (int i = 0; i < views; ++i) {
        V.rgb[i] = rgb[i];
        V.lev[i] = reinterpret_cast<float4 *>(levels[i]);
    }
    int64_t n0 = geoms[0].off[geoms[0].n_pairs];
    bool aligned = true;
    for (int i = 0; i < views; ++i) aligned = aligned && (reinterpret_cast<uintptr_t>(rgb[i]) & 3) == 0;
    if (aligned)
        k_level0_x4<<<dim3(grid_for((n0 + 3) / 4), views), kBlock, 0, st>>>(V, geoms[0]);
    else
        k_level0<<<dim3(grid_for(n0), views), kBlock, 0, st>>>(V, geoms[0]);
    for (int l = 0; l < L; ++l) {
        int64_t ni = geoms[l].off[geoms[l].n_pairs];
        int64_t no = geoms[l + 1].off[geoms[l + 1].n_pairs];
        for (int i = 0; i < views; ++i) {
            V.src[i] = V.lev[i];
            V.lev[i] = V.lev[i] + ni;
        }
        k_downsample<<<dim3(grid_for(no), views), kBlock, 0, st>>>(V, geoms[l], geoms[l + 1], S);
    }
}

void launch_predict_range(const int32_t *disp_up, const LevelGeom &gu, const LevelGeom &gl, int S,
                          int window, int32_t *lo, int32_t *hi, hipStream_t st) {
    int64_t n = gl.off[gl.n_pairs];
    k_predict_range<<<grid_for(n), kBlock, 0, st>>>(disp_up, gu, gl, S, window, lo, hi);
}

}  // namespace hdp
