// Host-side launchers of the HDP kernels (one translation unit per stage).
#pragma once

#include "common.hpp"

namespace hdp {

void launch_pyramid(const uint8_t *const *rgb, int views, const LevelGeom *geoms, int L, int S,
                    float *const *levels, hipStream_t st);
void launch_predict_range(const int32_t *disp_up, const LevelGeom &gu, const LevelGeom &gl, int S,
                          int window, int32_t *lo, int32_t *hi, hipStream_t st);

// Mixture model of one layer's label offsets, passed to kernels by value.
struct GmmParams {
    int K;
    double pi[HDP_MAX_GMM], mu[HDP_MAX_GMM], sd[HDP_MAX_GMM];
};
void launch_interval_table(const LevelGeom &gu, const LevelGeom &gl, int S, const GmmParams &m,
                           const double *prior, int prior_stride, double delta, int32_t *lo_tab,
                           int32_t *hi_tab, int tab_stride, int32_t *max_width, hipStream_t st);
// First sample centre of each pair and centres per row (sampled prior).
struct CentreTable {
    int64_t off[HDP_MAX_PAIRS + 1];
    int32_t nx[HDP_MAX_PAIRS];
};
void launch_mirror(const uint8_t *in, const LevelGeom &g, uint8_t *out, hipStream_t st);
void launch_lr_check(const int32_t *dl, const int32_t *dr, int right_mirrored, const LevelGeom &g,
                     int tol, uint8_t *stable, hipStream_t st);
void launch_sample_prior(const int32_t *disp, const uint8_t *stable, const LevelGeom &g,
                         int square, double *prior, int prior_stride, hipStream_t st);
void launch_refine_cost(const int32_t *disp, const uint8_t *stable, const hdp_forest &f,
                        int width, float *cost, hipStream_t st);
void launch_predict_range_table(const int32_t *disp_up, const LevelGeom &gu, const LevelGeom &gl,
                                int S, const int32_t *lo_tab, const int32_t *hi_tab,
                                int tab_stride, int32_t *lo, int32_t *hi, hipStream_t st);
void launch_cost_volume(const float *left, const float *right, const LevelGeom &g,
                        const int32_t *node, const int32_t *lo, const int32_t *hi, int width,
                        const hdp_cost_params &p, float *cost, hipStream_t st);
void launch_wta(const LevelGeom &g, const int32_t *node, const int32_t *lo, const int32_t *hi,
                int width, const float *agg, int32_t *disp, hipStream_t st);
size_t tree_workspace_bytes(int64_t n);
// literal: outside the exact regime, the sequential Kruskal process with both
// DT rules (beta_num / beta_den) instead of the minimum spanning forest.
void launch_build_tree(const float *img, const LevelGeom &g, const int32_t *plo,
                       const int32_t *phi, int max_width, int width, const int32_t *rank,
                       const hdp_forest &f, void *ws, hipStream_t st, bool literal = false,
                       int beta_num = 1, int beta_den = 1);
void launch_level_order(const hdp_forest &f, void *ws, hipStream_t st);
void launch_set_weights(const hdp_forest &f, const float *w, hipStream_t st);
size_t aggregate_workspace_bytes(int64_t n, int width);
bool set_schedule(int width, int cpt, int rpg);
void launch_aggregate(const hdp_forest &f, int width, const float *cost, float sigma, float *agg,
                      float *up, void *ws, hipStream_t st);
void launch_match(const float *left, const float *right, const LevelGeom &g, const hdp_forest &f,
                  int width, const hdp_cost_params &p, float sigma, float *agg, int32_t *disp,
                  void *ws, hipStream_t st);
void launch_aggregate_backward(const hdp_forest &f, int width, const float *cost, const float *agg,
                               const float *up, const float *grad_agg, float sigma,
                               float *grad_cost, float *grad_w, float *grad_sigma, void *ws,
                               hipStream_t st);

}  // namespace hdp
