// C ABI of the HDP library: host-side validation, batch geometry and dispatch
// to the HIP launchers.  Nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <cstring>

#include "hdp.h"
#include "kernels.hpp"

using hdp::LevelGeom;

namespace hdp {
namespace {
constexpr int kTimerSlots = 1024;
int g_timer_class = -1;
int g_timer_n = 0;
hipEvent_t g_ev[kTimerSlots][2];
bool g_ev_made = false;
}  // namespace

void timer_before(int kernel_class, hipStream_t st) {
    if (kernel_class != g_timer_class || g_timer_n >= kTimerSlots) return;
    (void)hipEventRecord(g_ev[g_timer_n][0], st);
}

void timer_after(int kernel_class, hipStream_t st) {
    if (kernel_class != g_timer_class || g_timer_n >= kTimerSlots) return;
    (void)hipEventRecord(g_ev[g_timer_n][1], st);
    ++g_timer_n;
}
}  // namespace hdp

namespace {

constexpr int64_t kMaxPixels = (int64_t(1) << 30) - 1;  // tour slot ids 4v+d below 2^32 - 1
constexpr int64_t kMaxPairPixels = (int64_t(1) << 22) - 1;  // packed depth field
// per-pixel arrays of up to 16-byte elements are addressed with 32-bit byte offsets
static_assert(HDP_MAX_PAIRS * kMaxPairPixels * 16 < (int64_t(1) << 32), "32-bit pixel offsets");

hdp_status last_hip() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HDP_OK : HDP_EHIP;
}

hdp_status make_geom(const hdp_shape *shapes, int32_t n_pairs, int32_t level, LevelGeom *g) {
    if (!shapes) return HDP_EINVAL;
    if (n_pairs < 1 || n_pairs > HDP_MAX_PAIRS) return HDP_ESHAPE;
    std::memset(g, 0, sizeof(*g));
    g->n_pairs = n_pairs;
    g->level = level;
    int64_t off = 0, toff = 0;
    for (int i = 0; i < n_pairs; ++i) {
        const hdp_shape &s = shapes[i];
        if (s.H < 1 || s.W < 1 || s.dmax < 0 || s.dmax >= HDP_MAX_LABELS) return HDP_ESHAPE;
        int64_t px = (int64_t)s.H * s.W;
        if (px > kMaxPairPixels) return HDP_ESHAPE;
        g->toff[i] = (int32_t)toff;
        toff += (int64_t)((s.H + hdp::kTile - 1) / hdp::kTile) * ((s.W + hdp::kTile - 1) / hdp::kTile);
        g->off[i] = (int32_t)off;
        g->H[i] = s.H;
        g->W[i] = s.W;
        g->dmax[i] = s.dmax;
        off += px;
        if (off > kMaxPixels) return HDP_ESHAPE;
    }
    g->off[n_pairs] = (int32_t)off;
    g->toff[n_pairs] = (int32_t)toff;
    return HDP_OK;
}

int64_t total_pixels(const LevelGeom &g) { return g.off[g.n_pairs]; }

int max_dmax(const LevelGeom &g) {
    int m = 0;
    for (int i = 0; i < g.n_pairs; ++i) m = g.dmax[i] > m ? g.dmax[i] : m;
    return m;
}

struct FLayout {
    size_t parent, depth, tree, lo, hi, row, wgt, order, level_ptr, node, prow, lc, heavy, rw,
        phase_ptr, info, rx, rlh, end;
};

FLayout forest_layout(int64_t n) {
    FLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        size_t at = off;
        off += bytes;
        return at;
    };
    L.parent = take(4 * n);
    L.depth = take(4 * n);
    L.tree = take(4 * n);
    L.lo = take(4 * n);
    L.hi = take(4 * n);
    L.row = take(4 * n);
    L.wgt = take(4 * n);
    L.order = take(4 * n);
    L.level_ptr = take(4 * (n + 1));
    L.node = take(4 * n);
    L.prow = take(4 * n);
    L.lc = take(4 * 2 * n);
    L.heavy = take(n);
    L.rw = take(4 * n);
    L.phase_ptr = take(4 * (HDP_MAX_PHASES + 1));
    L.info = take(4 * HDP_INFO_WORDS);
    L.rx = take(4 * n);
    L.rlh = take(4 * n);
    L.end = (off + 255) & ~size_t(255);
    return L;
}

bool forest_ok(const hdp_forest *f, int64_t n) {
    return f && f->n == n && f->parent && f->depth && f->tree && f->lo && f->hi && f->row &&
           f->wgt && f->order && f->level_ptr && f->node && f->prow && f->lc && f->heavy &&
           f->rw && f->phase_ptr && f->info && f->rx && f->rlh;
}

}  // namespace

extern "C" {

size_t hdp_forest_bytes(int64_t n) { return n < 1 ? 0 : forest_layout(n).end; }

hdp_status hdp_forest_bind(void *buf, size_t bytes, int64_t n, hdp_forest *f) {
    if (!buf || !f || n < 1) return HDP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(buf) & 255) != 0) return HDP_EINVAL;
    FLayout L = forest_layout(n);
    if (bytes < L.end) return HDP_EWORKSPACE;
    char *b = reinterpret_cast<char *>(buf);
    f->n = n;
    f->parent = reinterpret_cast<int32_t *>(b + L.parent);
    f->depth = reinterpret_cast<int32_t *>(b + L.depth);
    f->tree = reinterpret_cast<int32_t *>(b + L.tree);
    f->lo = reinterpret_cast<int32_t *>(b + L.lo);
    f->hi = reinterpret_cast<int32_t *>(b + L.hi);
    f->row = reinterpret_cast<int32_t *>(b + L.row);
    f->wgt = reinterpret_cast<float *>(b + L.wgt);
    f->order = reinterpret_cast<int32_t *>(b + L.order);
    f->level_ptr = reinterpret_cast<int32_t *>(b + L.level_ptr);
    f->node = reinterpret_cast<int32_t *>(b + L.node);
    f->prow = reinterpret_cast<int32_t *>(b + L.prow);
    f->lc = reinterpret_cast<int32_t *>(b + L.lc);
    f->heavy = reinterpret_cast<uint8_t *>(b + L.heavy);
    f->rw = reinterpret_cast<float *>(b + L.rw);
    f->phase_ptr = reinterpret_cast<int32_t *>(b + L.phase_ptr);
    f->info = reinterpret_cast<int32_t *>(b + L.info);
    f->rx = reinterpret_cast<int32_t *>(b + L.rx);
    f->rlh = reinterpret_cast<int32_t *>(b + L.rlh);
    return HDP_OK;
}

hdp_status hdp_level_shapes(const hdp_shape *shapes, int32_t n_pairs, int32_t S, int32_t L,
                            hdp_shape *out) {
    if (!shapes || !out) return HDP_EINVAL;
    if (n_pairs < 1 || n_pairs > HDP_MAX_PAIRS || S < 2 || L < 0 || L > 8) return HDP_ESHAPE;
    for (int i = 0; i < n_pairs; ++i) {
        hdp_shape s = shapes[i];
        if (s.H < 1 || s.W < 1 || s.dmax < 0) return HDP_ESHAPE;
        for (int l = 0; l <= L; ++l) {
            out[(size_t)l * n_pairs + i] = s;
            s.H = (s.H + S - 1) / S;
            s.W = (s.W + S - 1) / S;
            s.dmax = s.dmax / S;
        }
    }
    return HDP_OK;
}

static hdp_status pyramid_views(const uint8_t *const *rgb, int views, const hdp_shape *shapes,
                                int32_t n_pairs, int32_t S, int32_t L, float *const *levels,
                                void *stream) {
    for (int i = 0; i < views; ++i)
        if (!rgb[i] || !levels[i]) return HDP_EINVAL;
    if (S != 2 || L < 0 || L > 8) return HDP_EINVAL;
    hdp_shape ls[(8 + 1) * HDP_MAX_PAIRS];
    hdp_status st = hdp_level_shapes(shapes, n_pairs, S, L, ls);
    if (st != HDP_OK) return st;
    LevelGeom geoms[9];
    for (int l = 0; l <= L; ++l) {
        st = make_geom(ls + (size_t)l * n_pairs, n_pairs, l, &geoms[l]);
        if (st != HDP_OK) return st;
    }
    (void)hipGetLastError();
    hdp::launch_pyramid(rgb, views, geoms, L, S, levels, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_pyramid(const uint8_t *rgb, const hdp_shape *shapes, int32_t n_pairs, int32_t S,
                       int32_t L, float *levels, void *stream) {
    return pyramid_views(&rgb, 1, shapes, n_pairs, S, L, &levels, stream);
}

hdp_status hdp_pyramid_views(const uint8_t *left_rgb, const uint8_t *right_rgb,
                             const hdp_shape *shapes, int32_t n_pairs, int32_t S, int32_t L,
                             float *left_levels, float *right_levels, void *stream) {
    const uint8_t *rgb[2] = {left_rgb, right_rgb};
    float *levels[2] = {left_levels, right_levels};
    return pyramid_views(rgb, 2, shapes, n_pairs, S, L, levels, stream);
}

size_t hdp_build_tree_workspace_bytes(int64_t n) {
    return n < 1 ? 0 : hdp::tree_workspace_bytes(n);
}

static hdp_status build_tree(const float *img, const hdp_shape *shapes, int32_t n_pairs,
                             int32_t level, const int32_t *pix_lo, const int32_t *pix_hi,
                             int32_t max_width, int32_t beta_num, int32_t beta_den,
                             int32_t width, const int32_t *edge_rank, const hdp_forest *f,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!img || !ws) return HDP_EINVAL;
    if ((pix_lo == nullptr) != (pix_hi == nullptr)) return HDP_EINVAL;
    if (level < 0 || level > 8) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, level, &g);
    if (st != HDP_OK) return st;
    int64_t n = total_pixels(g);
    if (!forest_ok(f, n)) return HDP_EINVAL;
    if (width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    bool literal = false;
    if (pix_lo) {
        if (max_width < 1 || width < max_width) return HDP_EINVAL;
        if (beta_num < 1 || beta_den < 1 || beta_num > beta_den) return HDP_EINVAL;
        // exact regime: two distinct intervals of width <= w have IoU <= (w-1)/w < beta;
        // outside it the sequential process itself runs
        if ((int64_t)beta_num * max_width <= (int64_t)beta_den * (max_width - 1)) literal = true;
    } else if (width < max_dmax(g) + 1) {
        return HDP_EINVAL;
    }
    if (ws_bytes < hdp::tree_workspace_bytes(n)) return HDP_EWORKSPACE;
    (void)hipGetLastError();
    hdp::launch_build_tree(img, g, pix_lo, pix_hi, max_width, width, edge_rank, *f, ws,
                           (hipStream_t)stream, literal, beta_num, beta_den);
    return last_hip();
}

hdp_status hdp_build_tree(const float *img, const hdp_shape *shapes, int32_t n_pairs,
                          int32_t level, const int32_t *pix_lo, const int32_t *pix_hi,
                          int32_t max_width, int32_t beta_num, int32_t beta_den, int32_t width,
                          const hdp_forest *f, void *ws, size_t ws_bytes, void *stream) {
    return build_tree(img, shapes, n_pairs, level, pix_lo, pix_hi, max_width, beta_num, beta_den,
                      width, nullptr, f, ws, ws_bytes, stream);
}

hdp_status hdp_build_random_tree(const float *img, const hdp_shape *shapes, int32_t n_pairs,
                                 int32_t level, const int32_t *edge_rank, const int32_t *pix_lo,
                                 const int32_t *pix_hi, int32_t max_width, int32_t beta_num,
                                 int32_t beta_den, int32_t width, const hdp_forest *f, void *ws,
                                 size_t ws_bytes, void *stream) {
    if (!edge_rank) return HDP_EINVAL;
    return build_tree(img, shapes, n_pairs, level, pix_lo, pix_hi, max_width, beta_num, beta_den,
                      width, edge_rank, f, ws, ws_bytes, stream);
}

hdp_status hdp_level_order(const hdp_forest *f, void *ws, size_t ws_bytes, void *stream) {
    if (!f || !ws) return HDP_EINVAL;
    if (f->n < 1 || !forest_ok(f, f->n)) return HDP_EINVAL;
    if (ws_bytes < hdp::tree_workspace_bytes(f->n)) return HDP_EWORKSPACE;
    (void)hipGetLastError();
    hdp::launch_level_order(*f, ws, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_forest_read_info(const hdp_forest *f, int32_t *info_host, int32_t *phase_ptr_host,
                                void *stream) {
    if (!f || !f->info || !f->phase_ptr) return HDP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int32_t info[HDP_INFO_WORDS];
    if (hipMemcpyAsync(info, f->info, 4 * HDP_INFO_WORDS, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
        return HDP_EHIP;
    if (phase_ptr_host && hipMemcpyAsync(phase_ptr_host, f->phase_ptr, 4 * (HDP_MAX_PHASES + 1),
                                         hipMemcpyDeviceToHost, st) != hipSuccess)
        return HDP_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return HDP_EHIP;
    if (info_host) memcpy(info_host, info, sizeof(info));
    // a pixel interval that broke the caller's bound left an inexact forest
    return info[HDP_INFO_BAD_INTERVAL] > 0 ? HDP_EREGIME : HDP_OK;
}

hdp_status hdp_forest_set_weights(const hdp_forest *f, const float *wgt, void *stream) {
    if (!f || !wgt || f->n < 1 || !f->node || !f->parent || !f->wgt || !f->rw) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_set_weights(*f, wgt, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_cost_volume(const float *left, const float *right, const hdp_shape *shapes,
                           int32_t n_pairs, const hdp_forest *f, int32_t width,
                           const hdp_cost_params *p, float *cost, void *stream) {
    if (!left || !right || !p || !cost) return HDP_EINVAL;
    if (p->border != 0 && p->border != 1) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    int64_t n = total_pixels(g);
    if (f && !forest_ok(f, n)) return HDP_EINVAL;
    if (width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    if (!f && width < max_dmax(g) + 1) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_cost_volume(left, right, g, f ? f->node : nullptr, f ? f->lo : nullptr,
                            f ? f->hi : nullptr, width, *p, cost, (hipStream_t)stream);
    return last_hip();
}

size_t hdp_aggregate_workspace_bytes(int64_t n, int32_t width) {
    if (n < 1 || width < 1) return 0;
    return hdp::aggregate_workspace_bytes(n, width);
}

static hdp_status check_agg(const hdp_forest *f, int32_t width) {
    if (!f || !f->phase_ptr || !f->info || f->n < 1) return HDP_EINVAL;
    if (width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    if (f->n * (int64_t)width >= (int64_t(1) << 31)) return HDP_ESHAPE;  // 32-bit volume offsets
    return HDP_OK;
}

hdp_status hdp_aggregate(const hdp_forest *f, int32_t width, const float *cost, float sigma,
                         float *agg, float *up, void *ws, size_t ws_bytes, void *stream) {
    hdp_status st = check_agg(f, width);
    if (st != HDP_OK) return st;
    if (!cost || !agg || !ws || !(sigma > 0.f)) return HDP_EINVAL;
    if (ws_bytes < hdp::aggregate_workspace_bytes(f->n, width)) return HDP_EWORKSPACE;
    (void)hipGetLastError();
    hdp::launch_aggregate(*f, width, cost, sigma, agg, up, ws, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_match_layer(const float *left, const float *right, const hdp_shape *shapes,
                           int32_t n_pairs, const hdp_forest *f, int32_t width,
                           const hdp_cost_params *p, float sigma, float *agg, int32_t *disp,
                           void *ws, size_t ws_bytes, void *stream) {
    if (!left || !right || !p || !agg || !disp || !ws || !(sigma > 0.f)) return HDP_EINVAL;
    if (p->border != 0 && p->border != 1) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    if (!forest_ok(f, total_pixels(g))) return HDP_EINVAL;
    st = check_agg(f, width);
    if (st != HDP_OK) return st;
    if (ws_bytes < hdp::aggregate_workspace_bytes(f->n, width)) return HDP_EWORKSPACE;
    (void)hipGetLastError();
    hdp::launch_match(left, right, g, *f, width, *p, sigma, agg, disp, ws, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_aggregate_backward(const hdp_forest *f, int32_t width, const float *cost,
                                  const float *agg, const float *up, const float *grad_agg,
                                  float sigma, float *grad_cost, float *grad_w, float *grad_sigma,
                                  void *ws, size_t ws_bytes, void *stream) {
    hdp_status st = check_agg(f, width);
    if (st != HDP_OK) return st;
    if (!cost || !agg || !grad_agg || !grad_cost || !ws || !(sigma > 0.f)) return HDP_EINVAL;
    if (ws_bytes < hdp::aggregate_workspace_bytes(f->n, width)) return HDP_EWORKSPACE;
    (void)hipGetLastError();
    hdp::launch_aggregate_backward(*f, width, cost, agg, up, grad_agg, sigma, grad_cost, grad_w,
                                   grad_sigma, ws, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_wta(const hdp_forest *f, const hdp_shape *shapes, int32_t n_pairs, int32_t width,
                   const float *agg, int32_t *disp, void *stream) {
    if (!agg || !disp) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    int64_t n = total_pixels(g);
    if (f && !forest_ok(f, n)) return HDP_EINVAL;
    if (width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    if (!f && width < max_dmax(g) + 1) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_wta(g, f ? f->node : nullptr, f ? f->lo : nullptr, f ? f->hi : nullptr, width, agg,
                    disp, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_predict_range(const int32_t *disp_upper, const hdp_shape *upper,
                             const hdp_shape *lower, int32_t n_pairs, int32_t S, int32_t window,
                             int32_t *pix_lo, int32_t *pix_hi, void *stream) {
    if (!disp_upper || !pix_lo || !pix_hi) return HDP_EINVAL;
    if (S < 2 || window < 0) return HDP_EINVAL;
    LevelGeom gu, gl;
    hdp_status st = make_geom(upper, n_pairs, 1, &gu);
    if (st != HDP_OK) return st;
    st = make_geom(lower, n_pairs, 0, &gl);
    if (st != HDP_OK) return st;
    for (int i = 0; i < n_pairs; ++i) {
        if (gu.H[i] != (gl.H[i] + S - 1) / S || gu.W[i] != (gl.W[i] + S - 1) / S ||
            gu.dmax[i] != gl.dmax[i] / S)
            return HDP_ESHAPE;
    }
    (void)hipGetLastError();
    hdp::launch_predict_range(disp_upper, gu, gl, S, window, pix_lo, pix_hi, (hipStream_t)stream);
    return last_hip();
}

static hdp_status layer_pair_geoms(const hdp_shape *upper, const hdp_shape *lower,
                                   int32_t n_pairs, int32_t S, LevelGeom *gu, LevelGeom *gl) {
    if (S < 2) return HDP_EINVAL;
    hdp_status st = make_geom(upper, n_pairs, 1, gu);
    if (st != HDP_OK) return st;
    st = make_geom(lower, n_pairs, 0, gl);
    if (st != HDP_OK) return st;
    for (int i = 0; i < n_pairs; ++i) {
        if (gu->H[i] != (gl->H[i] + S - 1) / S || gu->W[i] != (gl->W[i] + S - 1) / S ||
            gu->dmax[i] != gl->dmax[i] / S)
            return HDP_ESHAPE;
    }
    return HDP_OK;
}

hdp_status hdp_interval_table(const hdp_shape *upper, const hdp_shape *lower, int32_t n_pairs,
                              int32_t S, const hdp_gmm *gmm, const double *prior,
                              int32_t prior_stride, double delta, int32_t *lo_tab,
                              int32_t *hi_tab, int32_t tab_stride, int32_t *max_width,
                              void *stream) {
    if (!gmm || !prior || !lo_tab || !hi_tab) return HDP_EINVAL;
    if (!(delta > 0.0 && delta <= 1.0)) return HDP_EINVAL;
    if (gmm->K < 1 || gmm->K > HDP_MAX_GMM) return HDP_EINVAL;
    hdp::GmmParams m{};
    m.K = gmm->K;
    for (int k = 0; k < gmm->K; ++k) {
        if (!(gmm->pi[k] >= 0.0) || !(gmm->sd[k] > 0.0) || !(gmm->mu[k] == gmm->mu[k]))
            return HDP_EINVAL;
        m.pi[k] = gmm->pi[k];
        m.mu[k] = gmm->mu[k];
        m.sd[k] = gmm->sd[k];
    }
    LevelGeom gu, gl;
    hdp_status st = layer_pair_geoms(upper, lower, n_pairs, S, &gu, &gl);
    if (st != HDP_OK) return st;
    for (int i = 0; i < n_pairs; ++i)
        if (prior_stride < gl.dmax[i] + 1 || tab_stride < gu.dmax[i] + 1) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_interval_table(gu, gl, S, m, prior, prior_stride, delta, lo_tab, hi_tab,
                               tab_stride, max_width, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_predict_range_table(const int32_t *disp_upper, const hdp_shape *upper,
                                   const hdp_shape *lower, int32_t n_pairs, int32_t S,
                                   const int32_t *lo_tab, const int32_t *hi_tab,
                                   int32_t tab_stride, int32_t *pix_lo, int32_t *pix_hi,
                                   void *stream) {
    if (!disp_upper || !lo_tab || !hi_tab || !pix_lo || !pix_hi) return HDP_EINVAL;
    LevelGeom gu, gl;
    hdp_status st = layer_pair_geoms(upper, lower, n_pairs, S, &gu, &gl);
    if (st != HDP_OK) return st;
    for (int i = 0; i < n_pairs; ++i)
        if (tab_stride < gu.dmax[i] + 1) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_predict_range_table(disp_upper, gu, gl, S, lo_tab, hi_tab, tab_stride, pix_lo,
                                    pix_hi, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_mirror(const uint8_t *rgb, const hdp_shape *shapes, int32_t n_pairs, uint8_t *out,
                      void *stream) {
    if (!rgb || !out || rgb == out) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    (void)hipGetLastError();
    hdp::launch_mirror(rgb, g, out, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_lr_check(const int32_t *disp_left, const int32_t *disp_right,
                        int32_t right_mirrored, const hdp_shape *shapes, int32_t n_pairs,
                        int32_t tol, uint8_t *stable, void *stream) {
    if (!disp_left || !disp_right || !stable || tol < 0) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    (void)hipGetLastError();
    hdp::launch_lr_check(disp_left, disp_right, right_mirrored != 0, g, tol, stable,
                         (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_sample_prior(const int32_t *disp, const uint8_t *stable, const hdp_shape *shapes,
                            int32_t n_pairs, int32_t square, double *prior, int32_t prior_stride,
                            void *stream) {
    if (!disp || !stable || !prior || square < 1) return HDP_EINVAL;
    LevelGeom g;
    hdp_status st = make_geom(shapes, n_pairs, 0, &g);
    if (st != HDP_OK) return st;
    if (prior_stride < max_dmax(g) + 1) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_sample_prior(disp, stable, g, square, prior, prior_stride, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_refine_cost(const int32_t *disp, const uint8_t *stable, const hdp_forest *f,
                           int32_t width, float *cost, void *stream) {
    if (!disp || !stable || !cost || !f || f->n < 1 || !f->node || !f->lo || !f->hi)
        return HDP_EINVAL;
    if (width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    (void)hipGetLastError();
    hdp::launch_refine_cost(disp, stable, *f, width, cost, (hipStream_t)stream);
    return last_hip();
}

hdp_status hdp_set_schedule(int32_t width, int32_t labels_per_thread, int32_t rows_per_group) {
    return hdp::set_schedule(width, labels_per_thread, rows_per_group) ? HDP_OK : HDP_EINVAL;
}

hdp_status hdp_timer_arm(int32_t kernel_class) {
    using namespace hdp;
    if (kernel_class >= 0 && !g_ev_made) {
        for (int i = 0; i < kTimerSlots; ++i)
            for (int k = 0; k < 2; ++k)
                if (hipEventCreate(&g_ev[i][k]) != hipSuccess) return HDP_EHIP;
        g_ev_made = true;
    }
    g_timer_class = kernel_class;
    g_timer_n = 0;
    return HDP_OK;
}

hdp_status hdp_timer_read(float *total_ms, int32_t *launches) {
    using namespace hdp;
    if (!total_ms || !launches) return HDP_EINVAL;
    float tot = 0.f;
    for (int i = 0; i < g_timer_n; ++i) {
        if (hipEventSynchronize(g_ev[i][1]) != hipSuccess) return HDP_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_ev[i][0], g_ev[i][1]) != hipSuccess) return HDP_EHIP;
        tot += ms;
    }
    *total_ms = tot;
    *launches = g_timer_n;
    return HDP_OK;
}

const char *hdp_status_str(hdp_status s) {
    switch (s) {
    case HDP_OK: return "ok";
    case HDP_EINVAL: return "invalid argument";
    case HDP_ESHAPE: return "invalid shape or batch";
    case HDP_EWORKSPACE: return "workspace too small";
    case HDP_EREGIME: return "beta and interval width outside the exact disparity-forest regime";
    case HDP_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

}  // extern "C"
