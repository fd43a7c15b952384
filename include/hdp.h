/*
 * hdp.h -- C ABI of the MI355X hot path of hierarchical-disparity-prediction
 * (HDP) stereo matching (Luo et al., "Fast Non-local Stereo Matching based on
 * Hierarchical Disparity Prediction").
 *
 * One layer of the method (Section 3) is
 *     hdp_predict_range  -> pixel intervals        (Section 3.1)
 *     hdp_build_tree     -> disparity forest       (Section 3.2)
 *     hdp_cost_volume    -> restricted cost E      (Section 3.3, eq. E)
 *     hdp_aggregate      -> aggregated cost C      (eq. W, eq. S, eq. C)
 *     hdp_wta            -> disparity map          (Section 3.3)
 * run top-down over the graph pyramid built by hdp_pyramid (Section 2.1).
 *
 * General rules
 *  - Every pointer argument is a DEVICE pointer unless stated otherwise; every
 *    call is asynchronous on `stream` (a hipStream_t, NULL = default stream).
 *  - The caller owns all memory.  No entry point allocates device memory;
 *    scratch space comes from a caller-provided workspace whose size is given
 *    by the matching *_workspace_bytes query.
 *  - A batch of `n_pairs` image pairs is processed by one call.  The pixels of
 *    the pairs are concatenated in pair order (pair p starts at the sum of
 *    H*W of the pairs before it); pixel (x, y) of a pair is at y*W + x.
 *    `shapes` is a HOST array of n_pairs entries, 1 <= n_pairs <= HDP_MAX_PAIRS.
 *  - Arguments are validated on the host before anything is enqueued; a call
 *    that returns an error has enqueued nothing.  A HIP runtime error seen
 *    while enqueueing is returned as HDP_EHIP.  No C++ exception crosses the
 *    ABI.
 *  - Labels are 0..dmax inclusive.
 *  - Size limits: each pair at most 2^22 - 1 pixels, a batch at most 2^30 - 1
 *    pixels per layer (HDP_ESHAPE otherwise).
 */
#ifndef HDP_H_
#define HDP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HDP_API __attribute__((visibility("default")))

#define HDP_MAX_PAIRS 64
#define HDP_MAX_LABELS 256   /* dmax + 1 <= 256 */
#define HDP_MAX_PHASES 40    /* bound on the chain phases of a forest */
#define HDP_INFO_WORDS 16

typedef enum {
    HDP_OK = 0,
    HDP_EINVAL = -1,      /* null pointer or out-of-range scalar */
    HDP_ESHAPE = -2,      /* bad image shape, dmax, or batch size */
    HDP_EWORKSPACE = -3,  /* workspace smaller than required */
    HDP_EREGIME = -4,     /* forest not exact: a pixel interval broke the bound given */
    HDP_EHIP = -5         /* HIP runtime error */
} hdp_status;

typedef struct {
    int32_t H, W;   /* image size in pixels */
    int32_t dmax;   /* largest label; labels are 0..dmax */
} hdp_shape;

typedef struct {
    float a_c, tau_c;   /* weight and truncation of the colour term */
    float a_g, tau_g;   /* weight and truncation of the gradient term */
    int32_t border;     /* a label d > x (the match falls left of the image):
                           0 = both terms at their truncation (default),
                           1 = compared with the row's first pixel;
                           the entry points taking these parameters return
                           HDP_EINVAL for any other value */
} hdp_cost_params;

/* Indices into hdp_forest.info (device int32 words written by hdp_build_tree). */
enum {
    HDP_INFO_N_LEVELS = 0,   /* 1 + largest depth (written by hdp_level_order) */
    HDP_INFO_N_PHASES = 1,   /* number of chain phases (1 + largest light depth) */
    HDP_INFO_N_TREES = 2,    /* number of trees in the forest */
    HDP_INFO_WIDTH = 3,      /* row width of the volume layout (labels per row) */
    HDP_INFO_MST_ROUNDS = 4, /* hooking rounds the spanning-forest build used */
    HDP_INFO_RANK_ROUNDS = 5,/* tour-ranking launches and LDS-tail rounds that advanced */
    HDP_INFO_BAD_INTERVAL = 6,/* pixels whose interval was empty or wider than allowed */
    HDP_INFO_ERROR = 7,      /* nonzero if an internal consistency guard tripped */
    HDP_INFO_LIVE_EDGES = 8, /* edges still joining two components after the tile-local phase */
    HDP_INFO_ACTIVE_COMPONENTS = 9, /* components with an edge left after the tile-local phase */
    HDP_INFO_TOUR_RUNS = 10, /* entries of the contracted Euler-tour list */
    HDP_INFO_LIST_EDGES = 11 /* edges still live after the full-grid rounds of the spanning
                                forest (0 when none ran or they finished it) */
};

/*
 * Disparity forest of one pyramid layer for a batch (Section 3.2), plus the
 * schedule that hdp_aggregate walks.  All arrays live inside ONE device
 * buffer owned by the caller: size it with hdp_forest_bytes(n) and carve it
 * with hdp_forest_bind (host-only, no GPU work).  n = total pixels of the
 * batch at this layer.
 *
 * Per pixel (pixel order):
 *   parent  parent pixel id, -1 at a root.  Each tree is rooted at its
 *           smallest pixel id.
 *   depth   edges from the root.
 *   tree    root pixel id of the pixel's tree.
 *   wgt     weight of the edge to the parent (max-channel |dI| / 255), 0 at
 *           roots.
 *   lo, hi  tree interval TreeIntv of the pixel's tree (labels).
 *   row     row of the pixel in the volume layout below.
 * Level order (canonical; written by hdp_level_order, not by hdp_build_tree,
 * and not used by the aggregation schedule):
 *   order   pixel ids sorted by (depth, id); level_ptr[k] = first position of
 *           depth k, level_ptr[n_levels] = n.  level_ptr has n + 1 entries.
 * Volume layout: a cost or aggregated volume is float[n][width]; row r holds
 * the labels lo(v) .. hi(v) of pixel v = node[r] at columns 0 .. hi-lo,
 * columns beyond are padding.  Rows are grouped in chain phases (heavy-path
 * decomposition): phase k = rows phase_ptr[k] .. phase_ptr[k+1]-1 hold the
 * pixels with k light edges on their root path; inside a phase every heavy
 * path is a contiguous run of rows, root side first.
 *   node    row -> pixel id.
 *   prow    row of the parent, -1 at roots.
 *   heavy   1 if the row's pixel is its parent's heavy child (same chain).
 *   lc      [2][n] rows of the light children, -1 where absent (a node has
 *           at most two: a tree is rooted at its smallest pixel id, whose
 *           upper and left neighbours lie outside its tree, so a root has at
 *           most two children and any other node at most three).
 *   rw      weight of the row's edge to its parent (= wgt[node]).
 *   rx      column (x) of the row's pixel in its image.
 *   rlh     interval of the row's pixel, lo | hi << 16 (= lo[node], hi[node]).
 *   phase_ptr  HDP_MAX_PHASES + 1 entries.
 *   info    HDP_INFO_WORDS device scalars (see HDP_INFO_*).
 */
typedef struct {
    int64_t n;
    int32_t *parent, *depth, *tree, *lo, *hi, *row;
    float *wgt;
    int32_t *order, *level_ptr;
    int32_t *node, *prow, *lc;
    uint8_t *heavy;
    float *rw;
    int32_t *phase_ptr, *info;
    int32_t *rx, *rlh;
} hdp_forest;

/* Bytes of the single device buffer that holds a forest of n pixels. */
HDP_API size_t hdp_forest_bytes(int64_t n);

/* Point the fields of *f into buf (host-only).  buf must be 256-byte aligned
 * and at least hdp_forest_bytes(n) long. */
HDP_API hdp_status hdp_forest_bind(void *buf, size_t bytes, int64_t n, hdp_forest *f);

/* Level shapes of the graph pyramid (Section 2.1): H_{l+1} = ceil(H_l / S),
 * W_{l+1} = ceil(W_l / S), d_{l+1} = floor(d_l / S).  out (HOST) receives
 * (L+1)*n_pairs shapes, level-major. */
HDP_API hdp_status hdp_level_shapes(const hdp_shape *shapes, int32_t n_pairs, int32_t S, int32_t L,
                            hdp_shape *out);

/*
 * Graph pyramid (Section 2.1) of one image per pair, S = 2 only.
 *   rgb     uint8 [n0][3] (interleaved RGB, the batch's pixels).
 *   levels  float [sum over l of n_l][4]: levels 0..L back to back; each
 *           pixel holds (R, G, B, gx) where R, G, B is the mean of the S x S
 *           nodes of the layer below that exist (exact in FP32 for S = 2) and
 *           gx = (R+G+B)(x+1) - (R+G+B)(x-1) with replicated borders, the
 *           numerator of the horizontal gray gradient used by the cost.
 */
HDP_API hdp_status hdp_pyramid(const uint8_t *rgb, const hdp_shape *shapes, int32_t n_pairs,
                       int32_t S, int32_t L, float *levels, void *stream);

/* The pyramids of both views of the batch (Section 2.1), in the same launches:
 * identical to hdp_pyramid on left_rgb -> left_levels and on right_rgb ->
 * right_levels. */
HDP_API hdp_status hdp_pyramid_views(const uint8_t *left_rgb, const uint8_t *right_rgb,
                                     const hdp_shape *shapes, int32_t n_pairs, int32_t S,
                                     int32_t L, float *left_levels, float *right_levels,
                                     void *stream);

/* Bytes of scratch space hdp_build_tree needs for n pixels. */
HDP_API size_t hdp_build_tree_workspace_bytes(int64_t n);

/*
 * Spanning tree (pix_lo == NULL: minimum spanning tree, Section 1 and
 * Rules 1-2 of Section 3.2) or disparity forest (DT-Rule 1 eq. cri1, DT-Rule 2
 * eq. DTrules) of one layer, with edge weight of eq. weight taken as the
 * largest channel difference.  Edges are ordered by (weight, edge id), edge id
 * 2p = right neighbour of p, 2p+1 = pixel below.
 *   img       level images as written by hdp_pyramid for this layer, [n][4].
 *   shapes    HOST shapes of this layer; level = pyramid layer (weights are
 *             exact integers at 4^level scale).
 *   pix_lo/hi pixel intervals PixelIntv (int32 [n]) or NULL for [0, dmax].
 *   max_width upper bound the caller guarantees on hi - lo + 1 (ignored when
 *             pix_lo is NULL).  When beta_num / beta_den > (max_width - 1) /
 *             max_width, DT-Rule 2 admits only equal intervals and the forest
 *             (the same as the sequential Kruskal process with both DT rules)
 *             is built as the minimum spanning forest of the equal-interval
 *             edges, in parallel.  The bound is checked on the device: pixels
 *             whose interval is empty, leaves [0, dmax] or is wider than
 *             max_width are counted in info[HDP_INFO_BAD_INTERVAL], their
 *             interval is clamped to [0, dmax] and max_width labels (so no later
 *             call reads or writes outside its buffers), the forest is then not
 *             the exact one, and hdp_forest_read_info returns HDP_EREGIME.
 *             Otherwise (outside that regime, e.g. beta = 3/5) the result
 *             depends on the order of the edges, and the sequential process
 *             itself runs on the device: the edges are sorted by (weight, id)
 *             and one workgroup takes them in that order (slow: one edge after
 *             another; meant for the small images that setting is used on).
 *             A tree's interval can then grow past max_width: `width` must
 *             hold the widest tree interval (dmax + 1 always does); a tree
 *             wider than `width`, or an empty or out-of-range pixel interval,
 *             is counted in info[HDP_INFO_BAD_INTERVAL].
 *   width     row width of the volume layout to prepare: at least the widest
 *             tree interval (dmax + 1 for the full range).
 */
HDP_API hdp_status hdp_build_tree(const float *img, const hdp_shape *shapes, int32_t n_pairs,
                          int32_t level, const int32_t *pix_lo, const int32_t *pix_hi,
                          int32_t max_width, int32_t beta_num, int32_t beta_den,
                          int32_t width, const hdp_forest *f, void *ws, size_t ws_bytes,
                          void *stream);

/*
 * Random spanning tree RT (Section 4.1: the edges are shuffled at random and
 * union-find keeps an edge when it joins two trees), or with pixel intervals
 * its disparity forest (HDP+RT, the DT rules applied in the shuffled order).
 *   edge_rank  int32 [2n] on the device, one random number per grid edge,
 *              drawn by the caller: edge_rank[2p] for the edge from pixel p
 *              to its right neighbour, edge_rank[2p+1] for the edge to the
 *              pixel below (entries of edges that leave the image are
 *              ignored).  Only the low 31 bits are used.  The shuffled order
 *              is ascending (rank, edge id); uniform random ranks give a
 *              uniformly random order of the edges up to ties.
 * Every other argument, the exact regime (outside it the sequential process
 * in the shuffled order), the outputs and the errors are those of
 * hdp_build_tree; the edge weights stored in the forest (and used by the
 * aggregation) are still the colour weights of eq. weight.  Returns
 * HDP_EINVAL if edge_rank is NULL.
 */
HDP_API hdp_status hdp_build_random_tree(const float *img, const hdp_shape *shapes,
                                         int32_t n_pairs, int32_t level,
                                         const int32_t *edge_rank, const int32_t *pix_lo,
                                         const int32_t *pix_hi, int32_t max_width,
                                         int32_t beta_num, int32_t beta_den, int32_t width,
                                         const hdp_forest *f, void *ws, size_t ws_bytes,
                                         void *stream);

/*
 * Canonical level order of a forest built by hdp_build_tree: order (pixel ids
 * sorted by depth, ties by id), level_ptr and info[HDP_INFO_N_LEVELS].  This
 * is the breadth-first processing order of the tree passes of Section 1; the
 * aggregation here runs on the chain-phase rows instead and does not need it.
 *   ws   scratch of at least hdp_build_tree_workspace_bytes(f->n) bytes.
 */
HDP_API hdp_status hdp_level_order(const hdp_forest *f, void *ws, size_t ws_bytes, void *stream);

/* Host copy of the forest's scalars and phase table (synchronises `stream`;
 * nothing on the hot path needs it).  Either pointer may be NULL;
 * phase_ptr_host receives HDP_MAX_PHASES + 1 entries.  Returns HDP_EREGIME
 * (after filling both outputs) when info[HDP_INFO_BAD_INTERVAL] > 0, i.e. the
 * forest was built from pixel intervals that broke hdp_build_tree's bounds (or,
 * outside the exact regime, a tree's interval outgrew the row width). */
HDP_API hdp_status hdp_forest_read_info(const hdp_forest *f, int32_t *info_host,
                                int32_t *phase_ptr_host, void *stream);

/*
 * Replace the forest's edge weights (eq. weight) by wgt[v] for the edge
 * (v, parent(v)), pixel order, float[n] (roots ignored): writes both the
 * per-pixel and the per-row copies.  Used to differentiate with respect to
 * learnable edge weights; the tree topology is unchanged.
 */
HDP_API hdp_status hdp_forest_set_weights(const hdp_forest *f, const float *wgt, void *stream);

/*
 * Restricted matching cost E (eq. E) of one layer.
 *   left/right  level images of the two views, [n][4] as written by
 *               hdp_pyramid.
 *   f           forest: cost is written in the forest's volume layout
 *               float[n][width] (width from hdp_build_tree);
 *               NULL: dense float[n][dmax+1] in pixel order, width = the
 *               largest dmax + 1 of the batch (a pair with a smaller range
 *               leaves its extra columns at 0).
 *   Entry (v, x) = a_c*min(mean_c |L_c(x,y) - R_c(x-d,y)|, tau_c)
 *                + a_g*min(|gx_L - gx_R| / 6, tau_g),
 *   and a_c*tau_c + a_g*tau_g where x - d < 0.  Padding columns are 0.
 */
HDP_API hdp_status hdp_cost_volume(const float *left, const float *right, const hdp_shape *shapes,
                           int32_t n_pairs, const hdp_forest *f, int32_t width,
                           const hdp_cost_params *p, float *cost, void *stream);

/* Bytes of scratch space hdp_aggregate / hdp_aggregate_backward need. */
HDP_API size_t hdp_aggregate_workspace_bytes(int64_t n, int32_t width);

/*
 * Tree aggregation (eq. W, eq. S, eq. C):
 *   agg(v, x) = sum over u in the tree of v of exp(-W(v,u)/sigma) * cost(u, x)
 * with W the sum of edge weights on the tree path, computed exactly by a
 * leaf-to-root and a root-to-leaf pass over the forest's chain phases (two
 * kernel launches; the phase table is read on the device, so the call never
 * synchronises with the host and can be captured in a HIP graph).
 *   cost, agg   float[n][width] in the forest's volume layout; width as given
 *               to hdp_build_tree (n * width < 2^31).
 *   up          optional (NULL) float[n][width]: receives the leaf-to-root
 *               sums U(v, x) = cost(v,x) + sum_children s_c U(c,x), which
 *               hdp_aggregate_backward can reuse instead of recomputing.
 *   sigma       > 0, the smoothing constant (sigma of eq. aggre / gamma of eq. S).
 * Internal consistency failures (never expected) set info[HDP_INFO_ERROR].
 */
HDP_API hdp_status hdp_aggregate(const hdp_forest *f, int32_t width, const float *cost,
                                 float sigma, float *agg, float *up, void *ws, size_t ws_bytes,
                                 void *stream);

/*
 * Adjoint of hdp_aggregate for L = sum g(v,x) agg(v,x), g = grad_agg:
 *   grad_cost = A^T g = A g (the aggregation operator is symmetric),
 *   grad_w[v] = dL/dw of the edge (v, parent(v)) in pixel order (0 at roots;
 *               NULL skips),
 *   grad_sigma (device, 1 float; NULL skips) = dL/dsigma.
 * cost/agg are the forward's input and output; up = the forward's U or NULL
 * (then it is recomputed from cost).  Same layout as hdp_aggregate.
 */
HDP_API hdp_status hdp_aggregate_backward(const hdp_forest *f, int32_t width, const float *cost,
                                          const float *agg, const float *up,
                                          const float *grad_agg, float sigma, float *grad_cost,
                                          float *grad_w, float *grad_sigma, void *ws,
                                          size_t ws_bytes, void *stream);

/*
 * Winner-takes-all (Section 3.3): disp[v] = the label of least aggregated cost
 * in [lo(v), hi(v)], lowest label on ties.
 *   f == NULL: agg is dense float[n][width] in pixel order, labels 0..dmax of
 *   each pair.  disp: int32 [n] in pixel order.
 */
HDP_API hdp_status hdp_wta(const hdp_forest *f, const hdp_shape *shapes, int32_t n_pairs,
                   int32_t width, const float *agg, int32_t *disp, void *stream);

/*
 * One layer's matching after the forest is built: restricted cost (Section
 * 3.3, eq. E), tree aggregation (eq. W, eq. S, eq. C) and winner-takes-all,
 * with the same results as hdp_cost_volume + hdp_aggregate + hdp_wta.  For
 * rows of at most 64 labels, or of up to 256 labels in multiples of four, the
 * up pass computes each row's cost from the level images as it goes (no cost
 * volume in memory; from 64 labels on it reads the right image packed in
 * 8 bytes a pixel, which the workspace holds, exactly where the pixels are
 * those of a pyramid of 2x2 means and as FP32 elsewhere) and the down pass
 * writes each row's winning label as its row is finished (no separate WTA
 * read of the aggregated volume); other rows run the three steps one after
 * another with the cost volume in the workspace.
 *   left, right, shapes, n_pairs, f, width, p: as hdp_cost_volume (f required).
 *   sigma       > 0, as hdp_aggregate.
 *   agg         float[n][width], receives the aggregated volume (volume layout).
 *   disp        int32[n] in pixel order, receives the labels.
 *   ws          hdp_aggregate_workspace_bytes(n, width) bytes of device memory.
 * Asynchronous on `stream`, never synchronises with the host, capturable.
 * Returns HDP_EINVAL for NULL arguments or a forest that does not match the
 * batch, HDP_EWORKSPACE for a short workspace.
 */
HDP_API hdp_status hdp_match_layer(const float *left, const float *right, const hdp_shape *shapes,
                           int32_t n_pairs, const hdp_forest *f, int32_t width,
                           const hdp_cost_params *p, float sigma, float *agg, int32_t *disp,
                           void *ws, size_t ws_bytes, void *stream);

/*
 * hdp_match_layer without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments (minus ws, ws_bytes),
 * same launches and the same results as hdp_match_layer.  Its scratch space
 * (the workspace of hdp_match_layer: coefficients, flags, tile maps, the U
 * volume) lives in one fixed device array of HDP_NOALLOC_SCRATCH_BYTES per
 * GPU, held from the library's load until the process ends; the call
 * allocates nothing.  Returns HDP_EWORKSPACE, enqueueing nothing, when
 * hdp_aggregate_workspace_bytes(f->n, width) exceeds that size (e.g. a layer
 * of up to about 2.4 million pixels at 10 labels per row fits).  Every call on
 * one GPU uses the same array and the kernels reinitialise what must start
 * clean, so calls in sequence are independent; calls that overlap on one GPU
 * (different streams or host threads) race on the array and must not be
 * issued.
 */
#define HDP_NOALLOC_SCRATCH_BYTES (256u << 20)
HDP_API size_t hdp_match_layer_noalloc_max_bytes(void);
HDP_API hdp_status hdp_match_layer_noalloc(const float *left, const float *right,
                                           const hdp_shape *shapes, int32_t n_pairs,
                                           const hdp_forest *f, int32_t width,
                                           const hdp_cost_params *p, float sigma, float *agg,
                                           int32_t *disp, void *stream);

/*
 * Pixel interval prediction (Section 3.1) for layer l from the disparity map
 * of layer l+1:
 *   PixelIntv(x, y) = [S*i - window, S*i + S - 1 + window] intersected with
 *   [0, dmax_l], i = disp_upper at (floor(x/S), floor(y/S)).
 * upper/lower are HOST shapes of layers l+1 and l (same pairs).
 * pix_lo/pix_hi: int32 [n_l].
 */
HDP_API hdp_status hdp_predict_range(const int32_t *disp_upper, const hdp_shape *upper,
                             const hdp_shape *lower, int32_t n_pairs, int32_t S,
                             int32_t window, int32_t *pix_lo, int32_t *pix_hi, void *stream);

/*
 * Bayesian pixel interval prediction (Section 2.2 eq. dpm, Section 3.1 eq.
 * crtr) for layer l of a batch, as a table over the parent's label.
 *   gmm        HOST pointer: the mixture model GMM_l of the offset
 *              o = D_{l+1} - floor(D_l / S): K components (1..HDP_MAX_GMM)
 *              with weights pi >= 0, means mu and standard deviations sd > 0
 *              (trained parameters; the paper does not print them).
 *   prior      device double [n_pairs][prior_stride]: the sampled
 *              distribution P(D_l = j) of each pair, j = 0..dmax_l (any
 *              non-negative scale; prior_stride >= every pair's dmax_l + 1).
 *   delta      threshold delta_l of eq. crtr (the paper uses
 *              delta_l = delta_0 * S^l), 0 < delta <= 1.
 *   lo_tab, hi_tab  device int32 [n_pairs][tab_stride] (tab_stride >= every
 *              pair's dmax_{l+1} + 1): the interval of parent label i.
 *   max_width  device int32 (1 word) or NULL: receives the widest interval.
 * Per pair and parent label i, with P(i, j) proportional to
 * GMM_l(i - floor(j/S)) * prior[j] and normalised over j = 0..dmax_l: the
 * interval starts at the label of highest P(i, j) (the lowest on ties) and
 * grows by its more probable neighbour label (the lower on ties) while
 * P / (c + P) >= delta, tested as P >= delta * (c + P) in FP64 with c the
 * probability selected so far; it stops at the first neighbour that fails.
 * A row whose products are all zero is taken without the prior; a row that is
 * still zero gets [S i, S i + S - 1] clipped to [0, dmax_l].
 * upper/lower: HOST shapes of layers l+1 and l, as hdp_predict_range.
 */
#define HDP_MAX_GMM 16
typedef struct {
    int32_t K;
    double pi[HDP_MAX_GMM], mu[HDP_MAX_GMM], sd[HDP_MAX_GMM];
} hdp_gmm;

HDP_API hdp_status hdp_interval_table(const hdp_shape *upper, const hdp_shape *lower,
                                      int32_t n_pairs, int32_t S, const hdp_gmm *gmm,
                                      const double *prior, int32_t prior_stride, double delta,
                                      int32_t *lo_tab, int32_t *hi_tab, int32_t tab_stride,
                                      int32_t *max_width, void *stream);

/*
 * Pixel intervals of layer l from a table (hdp_interval_table): pixel (x, y)
 * of a pair takes [lo_tab[i], hi_tab[i]] of that pair's row,
 * i = disp_upper at (floor(x/S), floor(y/S)).  pix_lo/pix_hi: int32 [n_l].
 */
HDP_API hdp_status hdp_predict_range_table(const int32_t *disp_upper, const hdp_shape *upper,
                                           const hdp_shape *lower, int32_t n_pairs, int32_t S,
                                           const int32_t *lo_tab, const int32_t *hi_tab,
                                           int32_t tab_stride, int32_t *pix_lo, int32_t *pix_hi,
                                           void *stream);

/*
 * Left-right consistency check and its uses (Section 3.1: the stable pixels
 * behind the sampled prior P(D_l); Section 3.3: the tree-based refinement that
 * can follow each layer).  The right view's labels are those of the method run
 * on the horizontally mirrored pair with the right image as reference.
 *
 * hdp_mirror: out(x, y) = rgb(W-1-x, y) for every pair, uint8 [n][3] (give it
 *   the right image for the reference view and the left image as the second
 *   view of the mirrored pair).
 * hdp_lr_check: stable[v] (uint8 0/1) for every pixel (x, y) of the left view
 *   with label d = disp_left[v]: 1 iff 0 <= x - d < W and
 *   |d - R| <= tol, R = the right view's label at column x - d, read from
 *   disp_right at column x - d, or at column W-1-(x-d) when right_mirrored is
 *   nonzero (disp_right is then the mirrored run's output as it stands).
 * hdp_sample_prior: prior (device double [n_pairs][prior_stride], overwritten)
 *   counts, per pair and label j = 0..dmax, the stable pixels among the
 *   centres (square/2 + k*square, square/2 + m*square) inside the image whose
 *   label is j (Section 3.1 uses square = 5).  prior_stride >= dmax + 1.
 * hdp_refine_cost: in the forest's volume layout float[n][width], the cost
 *   |x - disp[v]| of label x = lo(v) + c at a stable pixel v, 0 at an
 *   unstable one and in padding columns; hdp_aggregate + hdp_wta over the same
 *   forest then give the refined labels.
 * shapes: HOST shapes of the layer (n_pairs pairs).
 */
HDP_API hdp_status hdp_mirror(const uint8_t *rgb, const hdp_shape *shapes, int32_t n_pairs,
                              uint8_t *out, void *stream);
HDP_API hdp_status hdp_lr_check(const int32_t *disp_left, const int32_t *disp_right,
                                int32_t right_mirrored, const hdp_shape *shapes, int32_t n_pairs,
                                int32_t tol, uint8_t *stable, void *stream);
HDP_API hdp_status hdp_sample_prior(const int32_t *disp, const uint8_t *stable,
                                    const hdp_shape *shapes, int32_t n_pairs, int32_t square,
                                    double *prior, int32_t prior_stride, void *stream);
HDP_API hdp_status hdp_refine_cost(const int32_t *disp, const uint8_t *stable, const hdp_forest *f,
                                   int32_t width, float *cost, void *stream);

/*
 * Batch plan: the whole top-down loop of the method (Section 3) for a fixed
 * batch of pairs.  Layer L (the top of the graph pyramid) is searched over
 * [0, d_L] with the minimum spanning tree; every layer l < L predicts its pixel
 * intervals from layer l+1 (hdp_predict_range), builds the disparity forest,
 * the restricted cost, the aggregation and the WTA.
 * hdp_plan_create allocates every buffer once (this is the only place the
 * library allocates) and captures one step into a HIP graph; hdp_plan_run
 * copies the inputs (device pointers, uint8 [n0][3], NULL = already in the
 * plan's input buffers, see hdp_plan_inputs), launches the graph on `stream`
 * and copies the layer-0 labels to disp (device int32 [n0], NULL = skip).
 * Runs on one plan must not overlap.  Layer results stay readable through
 * hdp_plan_layer until the next run.
 */
typedef struct {
    int32_t S, L;                 /* pyramid factor (2) and layers above the input */
    int32_t window;               /* half-width w of the predicted interval */
    int32_t beta_num, beta_den;   /* DT-Rule 2 threshold beta = num/den */
    float sigma;                  /* smoothing constant */
    hdp_cost_params cost;
} hdp_params;

typedef struct hdp_plan_s *hdp_plan;

HDP_API hdp_status hdp_plan_create(const hdp_shape *shapes, int32_t n_pairs, const hdp_params *p,
                                   hdp_plan *out);
HDP_API hdp_status hdp_plan_run(hdp_plan plan, const uint8_t *left_rgb, const uint8_t *right_rgb,
                                int32_t *disp, void *stream);
HDP_API hdp_status hdp_plan_layer(hdp_plan plan, int32_t level, const hdp_forest **forest,
                                  const int32_t **disp, const float **agg, int32_t *width);
HDP_API hdp_status hdp_plan_inputs(hdp_plan plan, uint8_t **left_rgb, uint8_t **right_rgb);
HDP_API hdp_status hdp_plan_destroy(hdp_plan plan);

HDP_API const char *hdp_status_str(hdp_status s);

/*
 * Tile schedule of the aggregation passes for rows of `width` labels: each
 * thread handles `labels_per_thread` (1, 2 or 4; must divide width)
 * consecutive labels of `rows_per_group` (4, 8 or 16; 16 only with 2 labels
 * per thread) rows.  labels_per_thread = 0 restores the built-in
 * choice.  Process-wide host setting read when a pass is launched (a captured
 * graph keeps the schedule it was captured with); the workspace size does not
 * depend on it.  Set by the autotuner.
 */
HDP_API hdp_status hdp_set_schedule(int32_t width, int32_t labels_per_thread,
                                    int32_t rows_per_group);

/*
 * Diagnostics (not for use under graph capture): time every launch of one
 * kernel class with a pair of HIP events recorded on the launch's stream.
 * hdp_timer_arm(c) selects class c (or -1: off) and clears the record (at most
 * 1024 launches are kept); hdp_timer_read waits for the recorded events and
 * returns the summed kernel time in milliseconds and the number of launches.
 */
enum { HDP_TIMER_UP_PASS = 0, HDP_TIMER_DOWN_PASS = 1, HDP_TIMER_COST = 2 };
HDP_API hdp_status hdp_timer_arm(int32_t kernel_class);
HDP_API hdp_status hdp_timer_read(float *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* HDP_H_ */
