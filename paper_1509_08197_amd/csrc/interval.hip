// Bayesian pixel interval prediction (Section 2.2 eq. dpm, Section 3.1 eq. crtr).
//
// For one layer l and every pair of a batch, a table over the parent's label
// i = 0..d_{l+1}: the row P(D_l = j | D_{l+1} = i), proportional to
// GMM_l(i - floor(j/S)) * P(D_l = j) and normalised, gives the interval that
// starts at the row's most probable label and grows by its more probable
// neighbour label while eq. crtr holds.  Every pixel of layer l then takes the
// interval of its parent's label.
//
// The table decides integers from floating-point comparisons; it is computed
// in FP64 with no contraction, summing each row in ascending label order and
// taking each probability as (model * prior) / row sum, one thread per row.
#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

__device__ __forceinline__ double gauss_pdf(double o, double mu, double sd) {
#pragma clang fp contract(off)
    const double z = (o - mu) / sd;
    return exp(-0.5 * z * z) / (sd * 2.5066282746310002);  // sqrt(2 pi)
}

// GMM_l at offset o = i - floor(j / S).
__device__ __forceinline__ double gmm_at(const GmmParams &m, int o) {
#pragma clang fp contract(off)
    double q = 0.0;
    for (int k = 0; k < m.K; ++k) q += m.pi[k] * gauss_pdf((double)o, m.mu[k], m.sd[k]);
    return q;
}

__global__ void k_zero_word(int32_t *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// One thread per (pair, parent label i).
__global__ void __launch_bounds__(kBlock) k_interval_table(LevelGeom gu, LevelGeom gl, int S,
                                                           GmmParams m,
                                                           const double *__restrict__ prior,
                                                           int prior_stride, double delta,
                                                           int32_t *__restrict__ lo_tab,
                                                           int32_t *__restrict__ hi_tab,
                                                           int tab_stride, int32_t *max_width) {
#pragma clang fp contract(off)
    const int64_t t = gtid();
    const int pair = (int)(t / tab_stride), i = (int)(t - (int64_t)pair * tab_stride);
    if (pair >= gl.n_pairs || i > gu.dmax[pair]) return;
    const int dl = gl.dmax[pair];
    const double *pr = prior + (int64_t)pair * prior_stride;
    // probability of label j before normalisation (use_prior: with P(D_l))
    auto mass = [&](int j, bool use_prior) {
        const double q = gmm_at(m, i - j / S);
        return use_prior ? q * pr[j] : q;
    };
    bool use_prior = true;
    double tot = 0.0;
    for (int j = 0; j <= dl; ++j) tot += mass(j, true);
    if (tot == 0.0) {  // the prior has no mass where the model has: the model alone
        use_prior = false;
        for (int j = 0; j <= dl; ++j) tot += mass(j, false);
    }
    int lo, hi;
    if (tot == 0.0) {  // no information: the S labels below the parent's label
        lo = S * i > dl ? dl : S * i;
        hi = S * i + S - 1 > dl ? dl : S * i + S - 1;
    } else {
        int best = 0;
        double bp = mass(0, use_prior) / tot;
        for (int j = 1; j <= dl; ++j) {
            const double p = mass(j, use_prior) / tot;
            if (p > bp) {
                bp = p;
                best = j;
            }
        }
        lo = hi = best;
        double c = bp;
        double pl = lo > 0 ? mass(lo - 1, use_prior) / tot : 0.0;
        double ph = hi < dl ? mass(hi + 1, use_prior) / tot : 0.0;
        for (;;) {
            // the more probable neighbour (the lower one on ties)
            int cand = -1;
            double p = 0.0;
            if (lo > 0) {
                cand = lo - 1;
                p = pl;
            }
            if (hi < dl && (cand < 0 || ph > p)) {
                cand = hi + 1;
                p = ph;
            }
            if (cand < 0 || !(p >= delta * (c + p))) break;  // eq. crtr
            c += p;
            if (cand < lo) {
                lo = cand;
                pl = lo > 0 ? mass(lo - 1, use_prior) / tot : 0.0;
            } else {
                hi = cand;
                ph = hi < dl ? mass(hi + 1, use_prior) / tot : 0.0;
            }
        }
    }
    lo_tab[(int64_t)pair * tab_stride + i] = lo;
    hi_tab[(int64_t)pair * tab_stride + i] = hi;
    if (max_width) atomicMax(max_width, hi - lo + 1);
}

// Every pixel of layer l takes the interval of its parent's label.
__global__ void k_predict_range_table(const int32_t *__restrict__ disp_up, LevelGeom gu,
                                      LevelGeom gl, int S, const int32_t *__restrict__ lo_tab,
                                      const int32_t *__restrict__ hi_tab, int tab_stride,
                                      int32_t *__restrict__ lo, int32_t *__restrict__ hi) {
    const int64_t v = gtid();
    if (v >= gl.off[gl.n_pairs]) return;
    const PixelPos p = pixel_pos(gl, (int)v);
    const int i = disp_up[gu.off[p.pair] + (p.y / S) * gu.W[p.pair] + p.x / S];
    const int64_t k = (int64_t)p.pair * tab_stride + i;
    lo[v] = lo_tab[k];
    hi[v] = hi_tab[k];
}

void launch_interval_table(const LevelGeom &gu, const LevelGeom &gl, int S, const GmmParams &m,
                           const double *prior, int prior_stride, double delta, int32_t *lo_tab,
                           int32_t *hi_tab, int tab_stride, int32_t *max_width, hipStream_t st) {
    if (max_width) k_zero_word<<<1, 64, 0, st>>>(max_width);
    const int64_t n = (int64_t)gl.n_pairs * tab_stride;
    k_interval_table<<<grid_for(n), kBlock, 0, st>>>(gu, gl, S, m, prior, prior_stride, delta,
                                                     lo_tab, hi_tab, tab_stride, max_width);
}

void launch_predict_range_table(const int32_t *disp_up, const LevelGeom &gu, const LevelGeom &gl,
                                int S, const int32_t *lo_tab, const int32_t *hi_tab,
                                int tab_stride, int32_t *lo, int32_t *hi, hipStream_t st) {
    const int64_t n = gl.off[gl.n_pairs];
    k_predict_range_table<<<grid_for(n), kBlock, 0, st>>>(disp_up, gu, gl, S, lo_tab, hi_tab,
                                                          tab_stride, lo, hi);
}

}  // namespace hdp
