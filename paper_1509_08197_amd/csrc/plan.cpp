// Batch plan: the whole top-down HDP loop (Section 3) for a fixed batch of
// image pairs, with every buffer allocated once at creation and the step
// captured into one HIP graph, so that a run is a graph launch plus the input
// and output copies.  The plan is a client of the public C ABI.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "hdp.h"

namespace {

struct Level {
    std::vector<hdp_shape> shapes;
    int64_t n = 0;
    int width = 0;
    int max_width = 0;
    void *forest_buf = nullptr;
    hdp_forest forest{};
    int32_t *pix_lo = nullptr, *pix_hi = nullptr;
    float *agg = nullptr;
    int32_t *disp = nullptr;
    size_t level_off = 0;  // offset of this layer in the pyramid buffers (float4 units)
};

}  // namespace

struct hdp_plan_s {
    hdp_params p{};
    int n_pairs = 0;
    std::vector<hdp_shape> shapes;
    std::vector<Level> lv;
    int64_t n0 = 0;
    uint8_t *left = nullptr, *right = nullptr;
    float *lev_l = nullptr, *lev_r = nullptr;
    void *ws_tree = nullptr, *ws_agg = nullptr;
    size_t ws_tree_bytes = 0, ws_agg_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(hdp_plan_s *P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    for (Level &L : P->lv) {
        (void)hipFree(L.forest_buf);
        (void)hipFree(L.pix_lo);
        (void)hipFree(L.pix_hi);
        (void)hipFree(L.agg);
        (void)hipFree(L.disp);
    }
    (void)hipFree(P->left);
    (void)hipFree(P->right);
    (void)hipFree(P->lev_l);
    (void)hipFree(P->lev_r);
    (void)hipFree(P->ws_tree);
    (void)hipFree(P->ws_agg);
    delete P;
}

bool dev_alloc(void **p, size_t bytes) {
    return hipMalloc(p, bytes < 256 ? 256 : bytes) == hipSuccess;
}

// Enqueue one top-down step on stream st (no host synchronisation).
hdp_status enqueue_step(hdp_plan_s *P, hipStream_t st) {
    const hdp_params &p = P->p;
    hdp_status s = hdp_pyramid_views(P->left, P->right, P->shapes.data(), P->n_pairs, p.S, p.L,
                                     P->lev_l, P->lev_r, st);
    if (s != HDP_OK) return s;
    for (int l = p.L; l >= 0; --l) {
        Level &L = P->lv[l];
        const float *li = P->lev_l + 4 * L.level_off;
        const float *ri = P->lev_r + 4 * L.level_off;
        if (l < p.L) {
            Level &U = P->lv[l + 1];
            s = hdp_predict_range(U.disp, U.shapes.data(), L.shapes.data(), P->n_pairs, p.S,
                                  p.window, L.pix_lo, L.pix_hi, st);
            if (s != HDP_OK) return s;
        }
        s = hdp_build_tree(li, L.shapes.data(), P->n_pairs, l, l < p.L ? L.pix_lo : nullptr,
                           l < p.L ? L.pix_hi : nullptr, L.max_width, p.beta_num, p.beta_den,
                           L.width, &L.forest, P->ws_tree, P->ws_tree_bytes, st);
        if (s != HDP_OK) return s;
        s = hdp_match_layer(li, ri, L.shapes.data(), P->n_pairs, &L.forest, L.width, &p.cost,
                            p.sigma, L.agg, L.disp, P->ws_agg, P->ws_agg_bytes, st);
        if (s != HDP_OK) return s;
    }
    return HDP_OK;
}

}  // namespace

extern "C" {

hdp_status hdp_plan_create(const hdp_shape *shapes, int32_t n_pairs, const hdp_params *p,
                           hdp_plan *out) {
    if (!shapes || !p || !out) return HDP_EINVAL;
    *out = nullptr;
    if (n_pairs < 1 || n_pairs > HDP_MAX_PAIRS) return HDP_ESHAPE;
    if (p->S != 2 || p->L < 0 || p->L > 8 || p->window < 0 || !(p->sigma > 0.f)) return HDP_EINVAL;
    std::vector<hdp_shape> ls((size_t)(p->L + 1) * n_pairs);
    hdp_status s = hdp_level_shapes(shapes, n_pairs, p->S, p->L, ls.data());
    if (s != HDP_OK) return s;
    hdp_plan_s *P = new (std::nothrow) hdp_plan_s;
    if (!P) return HDP_EINVAL;
    P->p = *p;
    P->n_pairs = n_pairs;
    P->shapes.assign(shapes, shapes + n_pairs);
    P->lv.resize(p->L + 1);
    size_t lev_total = 0;
    int64_t max_n = 0;
    for (int l = 0; l <= p->L; ++l) {
        Level &L = P->lv[l];
        L.shapes.assign(ls.begin() + (size_t)l * n_pairs, ls.begin() + (size_t)(l + 1) * n_pairs);
        int dm = 0;
        for (const hdp_shape &sh : L.shapes) {
            L.n += (int64_t)sh.H * sh.W;
            dm = sh.dmax > dm ? sh.dmax : dm;
        }
        // top layer: full range [0, d_L]; below: the predicted window
        L.width = l == p->L ? dm + 1 : (p->S + 2 * p->window < dm + 1 ? p->S + 2 * p->window : dm + 1);
        L.max_width = l == p->L ? 0 : L.width;
        L.level_off = lev_total;
        lev_total += (size_t)L.n;
        max_n = L.n > max_n ? L.n : max_n;
    }
    P->n0 = P->lv[0].n;
    bool ok = dev_alloc((void **)&P->left, 3 * P->n0) && dev_alloc((void **)&P->right, 3 * P->n0) &&
              dev_alloc((void **)&P->lev_l, 16 * lev_total) &&
              dev_alloc((void **)&P->lev_r, 16 * lev_total);
    for (int l = 0; ok && l <= p->L; ++l) {
        Level &L = P->lv[l];
        size_t fb = hdp_forest_bytes(L.n);
        ok = dev_alloc(&L.forest_buf, fb) &&
             hdp_forest_bind(L.forest_buf, fb, L.n, &L.forest) == HDP_OK &&
             dev_alloc((void **)&L.pix_lo, 4 * L.n) && dev_alloc((void **)&L.pix_hi, 4 * L.n) &&
             dev_alloc((void **)&L.agg, 4 * L.n * L.width) && dev_alloc((void **)&L.disp, 4 * L.n);
        size_t wt = hdp_build_tree_workspace_bytes(L.n);
        size_t wa = hdp_aggregate_workspace_bytes(L.n, L.width);
        P->ws_tree_bytes = wt > P->ws_tree_bytes ? wt : P->ws_tree_bytes;
        P->ws_agg_bytes = wa > P->ws_agg_bytes ? wa : P->ws_agg_bytes;
    }
    ok = ok && dev_alloc(&P->ws_tree, P->ws_tree_bytes) && dev_alloc(&P->ws_agg, P->ws_agg_bytes);
    ok = ok && hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        free_plan(P);
        return HDP_EHIP;
    }
    // capture one step into a graph
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        free_plan(P);
        return HDP_EHIP;
    }
    s = enqueue_step(P, P->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap, &g);
    if (s != HDP_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        free_plan(P);
        return s != HDP_OK ? s : HDP_EHIP;
    }
    P->graph = g;
    if (hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        free_plan(P);
        return HDP_EHIP;
    }
    *out = P;
    return HDP_OK;
}

hdp_status hdp_plan_run(hdp_plan plan, const uint8_t *left_rgb, const uint8_t *right_rgb,
                        int32_t *disp, void *stream) {
    if (!plan) return HDP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hdp_plan_s *P = plan;
    if (left_rgb && left_rgb != P->left &&
        hipMemcpyAsync(P->left, left_rgb, 3 * P->n0, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HDP_EHIP;
    if (right_rgb && right_rgb != P->right &&
        hipMemcpyAsync(P->right, right_rgb, 3 * P->n0, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HDP_EHIP;
    if (hipGraphLaunch(P->exec, st) != hipSuccess) return HDP_EHIP;
    if (disp && hipMemcpyAsync(disp, P->lv[0].disp, 4 * P->n0, hipMemcpyDeviceToDevice, st) !=
                    hipSuccess)
        return HDP_EHIP;
    return HDP_OK;
}

hdp_status hdp_plan_layer(hdp_plan plan, int32_t level, const hdp_forest **forest,
                          const int32_t **disp, const float **agg, int32_t *width) {
    if (!plan || level < 0 || level > plan->p.L) return HDP_EINVAL;
    const Level &L = plan->lv[level];
    if (forest) *forest = &L.forest;
    if (disp) *disp = L.disp;
    if (agg) *agg = L.agg;
    if (width) *width = L.width;
    return HDP_OK;
}

hdp_status hdp_plan_inputs(hdp_plan plan, uint8_t **left_rgb, uint8_t **right_rgb) {
    if (!plan) return HDP_EINVAL;
    if (left_rgb) *left_rgb = plan->left;
    if (right_rgb) *right_rgb = plan->right;
    return HDP_OK;
}

hdp_status hdp_plan_destroy(hdp_plan plan) {
    free_plan(plan);
    return HDP_OK;
}

}  // extern "C"
