/*
 * hdp_oracle.c -- plain, slow, single-threaded FP64 CPU reference of the HDP
 * stereo hot path (Luo et al., "Fast Non-local Stereo Matching based on
 * Hierarchical Disparity Prediction").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the GPU library never calls it.
 *
 * Every function states the passage of the paper it follows.  Where the paper
 * is silent the reading used is stated at the function (the same readings are
 * listed in the design notes of the repository).
 *
 * Conventions
 *   - images are row-major (H, W, 3); pixel id p = y*W + x;
 *   - grid edge ids: 2p joins p and its right neighbour, 2p+1 joins p and the
 *     pixel below it (4-connected graph, Section 1 and Section 2.1);
 *   - labels are 0..dmax inclusive;
 *   - volumes are [pixel][label], entries outside a pixel's interval are NaN.
 *
 * Parity status: every exported function is pinned by the CPU tests against an
 * independent check (closed form, brute force, library routine or invariant).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Graph pyramid (Section 2.1): G_{l+1} merges S x S squares of G_l; the node
 * intensity is the average of the merged nodes; W_{l+1} = ceil(W_l / S),
 * H_{l+1} = ceil(H_l / S), d_{l+1} = floor(d_l / S).
 * Reading: where the image size is not a multiple of S the border squares hold
 * fewer than S^2 nodes and the average is taken over the nodes that exist. */

OR_API void or_level_dims(int H, int W, int dmax, int S, int L,
                          int32_t *Hs, int32_t *Ws, int32_t *dmaxs) {
    Hs[0] = H; Ws[0] = W; dmaxs[0] = dmax;
    for (int l = 0; l < L; ++l) {
        Hs[l + 1] = (Hs[l] + S - 1) / S;
        Ws[l + 1] = (Ws[l] + S - 1) / S;
        dmaxs[l + 1] = dmaxs[l] / S;
    }
}

/* out: levels 0..L concatenated, level l is (Hs[l], Ws[l], 3) doubles. */
OR_API void or_pyramid(const uint8_t *rgb, int H, int W, int S, int L, double *out) {
    int h = H, w = W;
    for (int i = 0; i < H * W * 3; ++i) out[i] = (double)rgb[i];
    double *prev = out;
    for (int l = 0; l < L; ++l) {
        int hn = (h + S - 1) / S, wn = (w + S - 1) / S;
        double *cur = prev + (size_t)h * w * 3;
        for (int Y = 0; Y < hn; ++Y)
            for (int X = 0; X < wn; ++X)
                for (int c = 0; c < 3; ++c) {
                    double sum = 0.0;
                    int cnt = 0;
                    for (int y = S * Y; y < S * Y + S && y < h; ++y)
                        for (int x = S * X; x < S * X + S && x < w; ++x) {
                            sum += prev[((size_t)y * w + x) * 3 + c];
                            ++cnt;
                        }
                    cur[((size_t)Y * wn + X) * 3 + c] = sum / cnt;
                }
        prev = cur; h = hn; w = wn;
    }
}

/* ------------------------------------------------------------------------ */
/* Pixel matching cost M(p, x) (Section 3.3, the cost used by E): truncated
 * absolute colour difference plus truncated difference of the horizontal
 * gradient.  The paper names the cost only by reference; reading:
 *   M = a_c * min(mean_c |I^L_c(x,y) - I^R_c(x-d,y)|, tau_c)
 *     + a_g * min(|gx^L(x,y) - gx^R(x-d,y)|, tau_g),
 *   gray g = (R+G+B)/3, gx(x) = (g(x+1) - g(x-1)) / 2 with replicated borders,
 *   and, when x-d falls left of the image, M = a_c*tau_c + a_g*tau_g (border
 *   policy 0, the reading used by default) or M against the row's first
 *   pixel (policy 1).
 * prm = {a_c, tau_c, a_g, tau_g, border}.  The gray difference is formed from
 * the channel sums, (sum(x+1) - sum(x-1)) / 6, which is the same quantity. */

static double chan_sum(const double *img, int W, int x, int y) {
    const double *p = img + ((size_t)y * W + x) * 3;
    return p[0] + p[1] + p[2];
}

static double gradx_num(const double *img, int W, int x, int y) {
    int xr = x + 1 < W ? x + 1 : W - 1;
    int xl = x - 1 >= 0 ? x - 1 : 0;
    return chan_sum(img, W, xr, y) - chan_sum(img, W, xl, y);
}

OR_API double or_matching_cost(const double *left, const double *right, int H, int W,
                               int x, int y, int d, const double *prm) {
    (void)H;
    int xr = x - d;
    if (xr < 0) {
        if (prm[4] == 0.0) return prm[0] * prm[1] + prm[2] * prm[3];
        xr = 0;
    }
    const double *pl = left + ((size_t)y * W + x) * 3;
    const double *pr = right + ((size_t)y * W + xr) * 3;
    double col = (fabs(pl[0] - pr[0]) + fabs(pl[1] - pr[1]) + fabs(pl[2] - pr[2])) / 3.0;
    double gd = fabs(gradx_num(left, W, x, y) - gradx_num(right, W, xr, y)) / 6.0;
    return prm[0] * fmin(col, prm[1]) + prm[2] * fmin(gd, prm[3]);
}

/* Restricted cost E (eq. E): M(p, x) for x inside the pixel's interval,
 * undefined (NaN) otherwise.  lo/hi NULL means the full range [0, dmax]. */
OR_API void or_cost_volume(const double *left, const double *right, int H, int W, int dmax,
                           const int32_t *lo, const int32_t *hi, const double *prm,
                           double *cost) {
    int D = dmax + 1;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int p = y * W + x;
            int a = lo ? lo[p] : 0, b = hi ? hi[p] : dmax;
            for (int d = 0; d < D; ++d)
                cost[(size_t)p * D + d] =
                    (d >= a && d <= b) ? or_matching_cost(left, right, H, W, x, y, d, prm) : NAN;
        }
}

/* ------------------------------------------------------------------------ */
/* Edge weights (eq. weight, Section 1): w(p,q) = |I(p) - I(q)|.  Reading: the
 * colour distance is the largest absolute channel difference, scaled by 1/255.
 * Level-l intensities are multiples of 4^-l (averages of 1, 2 or 4 nodes per
 * level with S = 2), so key = 4^l * max_c |dI_c| is an exact integer and
 * w = key / (255 * 4^l).  key < 0 marks an edge that leaves the image. */

OR_API void or_edge_keys(const double *img, int H, int W, int level, int64_t *key) {
    double scale = ldexp(1.0, 2 * level);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int p = y * W + x;
            for (int dir = 0; dir < 2; ++dir) {
                int q = dir == 0 ? (x + 1 < W ? p + 1 : -1) : (y + 1 < H ? p + W : -1);
                if (q < 0) { key[2 * p + dir] = -1; continue; }
                double m = 0.0;
                for (int c = 0; c < 3; ++c) {
                    double v = fabs(img[(size_t)p * 3 + c] - img[(size_t)q * 3 + c]);
                    if (v > m) m = v;
                }
                key[2 * p + dir] = (int64_t)llround(m * scale);
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Spanning tree / disparity forest by Kruskal (Section 3.2).
 *   Rule 1: take the remaining edge of least weight; ties broken by edge id
 *           (reading: the paper does not order equal weights).
 *   Rule 2: add it only if its ends lie in different trees (union-find).
 * HDP forest (pix_lo != NULL) adds:
 *   DT-Rule 1 (eq. cri1): discard the edge if the two pixel intervals are
 *           disjoint;
 *   DT-Rule 2 (eq. DTrules): merge two disparity trees only if
 *           |T_p n T_q| / |T_p u T_q| >= beta, tested exactly as
 *           beta_den*|n| >= beta_num*|u|; on merge T <- T_p u T_q.
 * Outputs: in_tree[2N] (1 if the edge is in the forest) and, per pixel, the
 * final interval of its tree (tree_lo/tree_hi, may be NULL).
 * Returns the number of forest edges. */

typedef struct { int64_t k; int32_t id; } or_edge;

static int cmp_edge(const void *a, const void *b) {
    const or_edge *x = (const or_edge *)a, *y = (const or_edge *)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int uf_find(int32_t *par, int v) {
    while (par[v] != v) { par[v] = par[par[v]]; v = par[v]; }
    return v;
}

OR_API int or_kruskal(int H, int W, const int64_t *key,
                      const int32_t *pix_lo, const int32_t *pix_hi,
                      int beta_num, int beta_den,
                      uint8_t *in_tree, int32_t *tree_lo, int32_t *tree_hi) {
    int N = H * W;
    or_edge *e = (or_edge *)malloc(sizeof(or_edge) * (size_t)2 * N);
    int ne = 0;
    for (int i = 0; i < 2 * N; ++i) {
        in_tree[i] = 0;
        if (key[i] >= 0) { e[ne].k = key[i]; e[ne].id = i; ++ne; }
    }
    qsort(e, ne, sizeof(or_edge), cmp_edge);
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *sz = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *tl = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *th = (int32_t *)malloc(sizeof(int32_t) * N);
    for (int v = 0; v < N; ++v) {
        par[v] = v; sz[v] = 1;
        tl[v] = pix_lo ? pix_lo[v] : 0;
        th[v] = pix_hi ? pix_hi[v] : 0;
    }
    int added = 0;
    for (int i = 0; i < ne; ++i) {
        int id = e[i].id, p = id >> 1, q = (id & 1) ? p + W : p + 1;
        if (pix_lo) {  /* DT-Rule 1 */
            int lo = pix_lo[p] > pix_lo[q] ? pix_lo[p] : pix_lo[q];
            int hi = pix_hi[p] < pix_hi[q] ? pix_hi[p] : pix_hi[q];
            if (lo > hi) continue;
        }
        int rp = uf_find(par, p), rq = uf_find(par, q);
        if (rp == rq) continue;  /* Rule 2 */
        if (pix_lo) {  /* DT-Rule 2 on the current tree intervals */
            int ilo = tl[rp] > tl[rq] ? tl[rp] : tl[rq];
            int ihi = th[rp] < th[rq] ? th[rp] : th[rq];
            int64_t inter = ihi >= ilo ? (int64_t)(ihi - ilo + 1) : 0;
            int64_t uni = (int64_t)(th[rp] - tl[rp] + 1) + (th[rq] - tl[rq] + 1) - inter;
            if ((int64_t)beta_den * inter < (int64_t)beta_num * uni) continue;
        }
        /* merge (union by size); the union of two intersecting intervals */
        if (sz[rp] < sz[rq]) { int t = rp; rp = rq; rq = t; }
        par[rq] = rp; sz[rp] += sz[rq];
        if (tl[rq] < tl[rp]) tl[rp] = tl[rq];
        if (th[rq] > th[rp]) th[rp] = th[rq];
        in_tree[id] = 1;
        ++added;
    }
    if (tree_lo && tree_hi)
        for (int v = 0; v < N; ++v) {
            int r = uf_find(par, v);
            tree_lo[v] = tl[r]; tree_hi[v] = th[r];
        }
    free(e); free(par); free(sz); free(tl); free(th);
    return added;
}

/* ------------------------------------------------------------------------ */
/* Rooting and level order.  The paper does not fix a root or an order
 * (aggregated values do not depend on them).  Reading: each tree is rooted at
 * its smallest pixel id; depth counts edges from the root; the level order
 * lists nodes by (depth, pixel id); level_ptr[k] is the first position of
 * depth k.  parent = -1 at roots; wgt is the weight of the edge to the parent
 * (0 at roots); tree holds the root id.  Returns the number of levels. */

static int nbr_edge(int H, int W, int v, int k, int *q) {
    int x = v % W, y = v / W;
    switch (k) {
    case 0: if (x + 1 < W) { *q = v + 1; return 2 * v; } break;
    case 1: if (y + 1 < H) { *q = v + W; return 2 * v + 1; } break;
    case 2: if (x > 0) { *q = v - 1; return 2 * (v - 1); } break;
    case 3: if (y > 0) { *q = v - W; return 2 * (v - W) + 1; } break;
    }
    return -1;
}

OR_API int or_root_forest(int H, int W, const uint8_t *in_tree, const int64_t *key, int level,
                          int32_t *parent, double *wgt, int32_t *depth, int32_t *tree,
                          int32_t *order, int32_t *level_ptr) {
    int N = H * W;
    double wscale = 255.0 * ldexp(1.0, 2 * level);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * N);
    for (int v = 0; v < N; ++v) parent[v] = -2;  /* unvisited */
    int maxd = 0;
    for (int r = 0; r < N; ++r) {
        if (parent[r] != -2) continue;
        parent[r] = -1; depth[r] = 0; wgt[r] = 0.0; tree[r] = r;
        int sp = 0;
        stack[sp++] = r;
        while (sp) {
            int v = stack[--sp];
            for (int k = 0; k < 4; ++k) {
                int q, id = nbr_edge(H, W, v, k, &q);
                if (id < 0 || !in_tree[id] || q == parent[v]) continue;
                parent[q] = v; depth[q] = depth[v] + 1; tree[q] = r;
                wgt[q] = (double)key[id] / wscale;
                if (depth[q] > maxd) maxd = depth[q];
                stack[sp++] = q;
            }
        }
    }
    int nl = maxd + 1;
    for (int k = 0; k <= nl; ++k) level_ptr[k] = 0;
    for (int v = 0; v < N; ++v) level_ptr[depth[v] + 1]++;
    for (int k = 0; k < nl; ++k) level_ptr[k + 1] += level_ptr[k];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (nl + 1));
    memcpy(fill, level_ptr, sizeof(int32_t) * (nl + 1));
    for (int v = 0; v < N; ++v) order[fill[depth[v]]++] = v;  /* ids ascending */
    free(fill); free(stack);
    return nl;
}

/* ------------------------------------------------------------------------ */
/* Aggregation, plain definition (eq. aggre with w_ij = exp(-D(i,j)/sigma),
 * and eq. W / eq. S / eq. C): for every listed pixel p,
 *   agg(p, x) = sum over q in the tree of p of exp(-W(p,q)/gamma) * C(q, x),
 * where W(p,q) is the sum of edge weights on the tree path.  sigma = gamma
 * (reading: one smoothing constant).  Unnormalised, as in eq. C.
 * edge_w[2N] are the grid-edge weights; in_tree selects the forest edges.
 * cost is [N][D] (NaN entries are skipped: undefined costs of eq. E).
 * out is [n_pix][D]. */

OR_API void or_aggregate_direct(int H, int W, const uint8_t *in_tree, const double *edge_w,
                                double sigma, int D, const double *cost,
                                const int32_t *pixels, int n_pix, double *out) {
    int N = H * W;
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *from = (int32_t *)malloc(sizeof(int32_t) * N);
    double *plen = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < n_pix; ++i) {
        int p = pixels[i];
        double *o = out + (size_t)i * D;
        for (int d = 0; d < D; ++d) o[d] = 0.0;
        int sp = 0;
        stack[sp++] = p; from[p] = -1; plen[p] = 0.0;
        while (sp) {
            int v = stack[--sp];
            double s = exp(-plen[v] / sigma);
            const double *c = cost + (size_t)v * D;
            for (int d = 0; d < D; ++d)
                if (!isnan(c[d])) o[d] += s * c[d];
            for (int k = 0; k < 4; ++k) {
                int q, id = nbr_edge(H, W, v, k, &q);
                if (id < 0 || !in_tree[id] || q == from[v]) continue;
                from[q] = v; plen[q] = plen[v] + edge_w[id];
                stack[sp++] = q;
            }
        }
        const double *cp = cost + (size_t)p * D;
        for (int d = 0; d < D; ++d)
            if (isnan(cp[d])) o[d] = NAN;
    }
    free(stack); free(from); free(plen);
}

/* Aggregation by the linear-time two-pass algorithm that the tree methods use
 * (Section 1: an exact algorithm with a leaf-to-root and a root-to-leaf pass).
 * With s_v = exp(-w(v, parent)/sigma):
 *   up   (deepest level first): U(v) = C(v) + sum_{children c} s_c * U(c)
 *   down (root first):          A(root) = U(root),
 *                               A(v) = s_v * A(parent) + (1 - s_v^2) * U(v).
 * U(v) collects the subtree of v; A(parent) - s_v U(v) is what the parent
 * receives from outside that subtree, so A(v) = U(v) + s_v (A(p) - s_v U(v)),
 * the same sum as the plain definition.  cost/agg are [N][D]; NaN entries are
 * carried through (they only meet entries of the same tree).  up (may be NULL)
 * receives U. */

OR_API void or_aggregate_twopass(int N, const int32_t *parent, const double *wgt,
                                 const int32_t *order, double sigma, int D,
                                 const double *cost, double *agg, double *up) {
    double *U = (double *)malloc(sizeof(double) * (size_t)N * D);
    memcpy(U, cost, sizeof(double) * (size_t)N * D);
    for (int i = N - 1; i >= 0; --i) {
        int v = order[i], p = parent[v];
        if (p < 0) continue;
        double s = exp(-wgt[v] / sigma);
        for (int d = 0; d < D; ++d) U[(size_t)p * D + d] += s * U[(size_t)v * D + d];
    }
    for (int i = 0; i < N; ++i) {
        int v = order[i], p = parent[v];
        if (p < 0) {
            for (int d = 0; d < D; ++d) agg[(size_t)v * D + d] = U[(size_t)v * D + d];
            continue;
        }
        double s = exp(-wgt[v] / sigma);
        for (int d = 0; d < D; ++d)
            agg[(size_t)v * D + d] = s * agg[(size_t)p * D + d] + (1.0 - s * s) * U[(size_t)v * D + d];
    }
    if (up) memcpy(up, U, sizeof(double) * (size_t)N * D);
    free(U);
}

/* ------------------------------------------------------------------------ */
/* Winner-takes-all (Section 3.3): the label of least aggregated cost inside
 * the pixel's interval.  Reading: ties go to the lowest label.  c1/c2 (may be
 * NULL) receive the best and second-best costs (c2 = +inf if the interval has
 * a single label). */

OR_API void or_wta(int N, int D, const double *agg, const int32_t *lo, const int32_t *hi,
                   int32_t *disp, double *c1, double *c2) {
    for (int p = 0; p < N; ++p) {
        int a = lo ? lo[p] : 0, b = hi ? hi[p] : D - 1;
        int best = a;
        double bv = agg[(size_t)p * D + a], sv = INFINITY;
        for (int d = a + 1; d <= b; ++d) {
            double v = agg[(size_t)p * D + d];
            if (v < bv) { sv = bv; bv = v; best = d; }
            else if (v < sv) sv = v;
        }
        disp[p] = best;
        if (c1) c1[p] = bv;
        if (c2) c2[p] = sv;
    }
}

/* ------------------------------------------------------------------------ */
/* Pixel interval prediction (Section 3.1).  The top layer uses [0, d_L].  For
 * a lower layer the paper derives the interval from a trained mixture model;
 * reading used here: a window of half-width w around the S x S block of labels
 * that maps to the parent's label i = D_{l+1}(floor(x/S), floor(y/S)):
 *   PixelIntv = [S*i - w, S*i + S - 1 + w] intersected with [0, d_l]. */

OR_API void or_predict_range(const int32_t *disp_up, int Hu, int Wu, int H, int W, int S,
                             int window, int dmax_l, int32_t *lo, int32_t *hi) {
    (void)Hu;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int i = disp_up[(y / S) * Wu + (x / S)];
            int a = S * i - window, b = S * i + S - 1 + window;
            lo[y * W + x] = a < 0 ? 0 : a;
            hi[y * W + x] = b > dmax_l ? dmax_l : b;
        }
}

/* ------------------------------------------------------------------------ */
/* Bayesian pixel interval prediction (Section 2.2 eq. dpm, Section 3.1 eq.
 * crtr), as a table over the parent's label i = 0..d_up for one layer l with
 * labels 0..dl:
 *   1. P(D_{l+1}=i | D_l=j) = GMM_l(i - floor(j/S)),
 *      GMM_l(o) = sum_k pi_k N(o | mu_k, sd_k) (Section 2.2);
 *   2. P(D_l=j | D_{l+1}=i) is proportional to P(D_{l+1}=i | D_l=j) P(D_l=j)
 *      (eq. dpm, prior[j] = the sampled distribution P(D_l=j), any scale),
 *      each row i normalised to sum 1 (Section 3.1);
 *   3. the interval starts at the label of highest probability in row i and is
 *      extended by a label j while P(i,j) / (c + P(i,j)) >= delta, c the
 *      probability already selected (eq. crtr).
 * Readings (the paper leaves them open): ties of the argmax go to the lowest
 * label; the interval grows by one of its two neighbour labels at a time, the
 * more probable one (the lower on ties), and stops at the first neighbour that
 * fails the test (the other one, no more probable, would fail too), so the
 * result is an interval; the test is evaluated as p >= delta * (c + p).  A row
 * whose products are all zero carries no information from the prior: it is
 * taken without the prior (uniform P(D_l)); a row that is still zero gets the
 * S labels below the parent's label, [S i, S i + S - 1] clipped to [0, dl]. */

static double or_gauss(double o, double mu, double sd) {
    double z = (o - mu) / sd;
    return exp(-0.5 * z * z) / (sd * 2.5066282746310002);  /* sqrt(2 pi) */
}

OR_API void or_gmm_interval_table(int S, int dl, int d_up, int K, const double *pi,
                                  const double *mu, const double *sd, const double *prior,
                                  double delta, int32_t *lo_tab, int32_t *hi_tab) {
    double *row = (double *)malloc(sizeof(double) * (size_t)(dl + 1));
    for (int i = 0; i <= d_up; ++i) {
        double tot = 0.0;
        for (int pass = 0; pass < 2 && tot == 0.0; ++pass) {
            tot = 0.0;
            for (int j = 0; j <= dl; ++j) {
                double q = 0.0;
                for (int k = 0; k < K; ++k) q += pi[k] * or_gauss((double)(i - j / S), mu[k], sd[k]);
                row[j] = pass == 0 ? q * prior[j] : q;
                tot += row[j];
            }
        }
        if (tot == 0.0) {
            int a = S * i > dl ? dl : S * i, b = S * i + S - 1 > dl ? dl : S * i + S - 1;
            lo_tab[i] = a; hi_tab[i] = b;
            continue;
        }
        int best = 0;
        for (int j = 0; j <= dl; ++j) {
            row[j] /= tot;
            if (row[j] > row[best]) best = j;
        }
        int lo = best, hi = best;
        double c = row[best];
        for (;;) {
            int cand = -1;
            if (lo > 0) cand = lo - 1;
            if (hi < dl && (cand < 0 || row[hi + 1] > row[cand])) cand = hi + 1;
            if (cand < 0) break;
            double p = row[cand];
            if (!(p >= delta * (c + p))) break;
            c += p;
            if (cand < lo) lo = cand; else hi = cand;
        }
        lo_tab[i] = lo; hi_tab[i] = hi;
    }
    free(row);
}

/* Interval of every pixel of layer l from the table of its parent's label:
 * PixelIntv(x, y) = [lo_tab[i], hi_tab[i]], i = D_{l+1}(floor(x/S), floor(y/S)). */
OR_API void or_predict_range_table(const int32_t *disp_up, int Hu, int Wu, int H, int W, int S,
                                   const int32_t *lo_tab, const int32_t *hi_tab, int32_t *lo,
                                   int32_t *hi) {
    (void)Hu;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int i = disp_up[(y / S) * Wu + (x / S)];
            lo[y * W + x] = lo_tab[i];
            hi[y * W + x] = hi_tab[i];
        }
}

/* ------------------------------------------------------------------------ */
/* Left-right consistency check: the stable pixels of Section 3.1 (found "by
 * left-to-right consistency check" as in the cited refinement method).  A
 * left-view pixel (x, y) with label d is stable when its match x - d lies in
 * the image and the right view's label there differs from d by at most tol.
 * Reading: the right view's labels come from the same method run on the
 * horizontally mirrored pair with the right image as reference; disp_r_mir is
 * that run's output in mirrored coordinates, so the right view's label of
 * column x is disp_r_mir at column W-1-x.  tol = 0 (equal labels) is the
 * usual check. */

OR_API void or_lr_check(const int32_t *disp_l, const int32_t *disp_r_mir, int H, int W, int tol,
                        uint8_t *stable) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int d = disp_l[y * W + x], xr = x - d;
            int ok = 0;
            if (xr >= 0 && xr < W) {
                int dr = disp_r_mir[y * W + (W - 1 - xr)];
                ok = (d - dr <= tol) && (dr - d <= tol);
            }
            stable[y * W + x] = (uint8_t)ok;
        }
}

/* Sampled distribution P(D_l) (Section 3.1): the layer is cut into
 * square x square blocks and the labels of the blocks' centres that are
 * stable are counted, prior[j] = number of such centres with label j.
 * Reading: the centres are (square/2 + k*square) in both directions, those
 * inside the image (a partial border block whose centre falls outside is not
 * sampled). */

OR_API void or_sample_prior(const int32_t *disp, const uint8_t *stable, int H, int W, int square,
                            int dmax, double *prior) {
    for (int j = 0; j <= dmax; ++j) prior[j] = 0.0;
    for (int y = square / 2; y < H; y += square)
        for (int x = square / 2; x < W; x += square) {
            int p = y * W + x;
            if (!stable[p]) continue;
            int d = disp[p];
            if (d >= 0 && d <= dmax) prior[d] += 1.0;
        }
}

/* Cost of the tree-based refinement that Section 3.3 says can be added after
 * each layer (the non-local refinement of the cited tree methods): a stable
 * pixel p costs |x - D(p)| at label x, an unstable one costs 0, so that after
 * aggregating over the same forest every pixel is pulled towards the labels of
 * the stable pixels near it on the tree.  cost[N][dmax+1]; entries outside a
 * pixel's [lo, hi] (lo/hi may be NULL for the full range) are NaN. */

OR_API void or_refine_cost(const int32_t *disp, const uint8_t *stable, int N, int dmax,
                           const int32_t *lo, const int32_t *hi, double *cost) {
    for (int p = 0; p < N; ++p)
        for (int x = 0; x <= dmax; ++x) {
            double *c = cost + (size_t)p * (dmax + 1) + x;
            if (lo && (x < lo[p] || x > hi[p])) { *c = NAN; continue; }
            *c = stable[p] ? fabs((double)(x - disp[p])) : 0.0;
        }
}

/* ------------------------------------------------------------------------ */
/* One layer of the method (Section 3): forest over the layer's graph, E over
 * each tree interval, aggregation over the forest and winner-takes-all,
 * one label slice at a time so that memory stays O(N).
 *   pix_lo == NULL: full range [0, dmax] and the plain MST (Rules 1-2 only).
 * Optional outputs (NULL to skip): parent, depth, order, level_ptr, tree_lo,
 * tree_hi, c1, c2 (see or_wta), and sampled aggregated slices
 * sample_agg[n_sample][N] at labels sample_d (NaN outside a tree interval).
 * rank == NULL: Kruskal takes the edges by colour weight (MST, DT).  Otherwise
 * rank[2N] holds one random number per grid edge (drawn by the caller) and the
 * edges are taken in ascending (rank, id) order: the random spanning tree (RT)
 * of Section 4.1 and its HDP forest.
 * Returns the number of levels of the forest. */

OR_API int or_stereo_level(const double *left, const double *right, int H, int W, int dmax,
                           int level, const int32_t *pix_lo, const int32_t *pix_hi,
                           int beta_num, int beta_den, double sigma, const double *prm,
                           int32_t *disp, double *c1, double *c2,
                           int32_t *parent_o, int32_t *depth_o, int32_t *order_o,
                           int32_t *level_ptr_o, int32_t *tree_lo_o, int32_t *tree_hi_o,
                           int n_sample, const int32_t *sample_d, double *sample_agg,
                           const int64_t *rank) {
    int N = H * W;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)2 * N);
    int64_t *order_key = (int64_t *)malloc(sizeof(int64_t) * (size_t)2 * N);
    uint8_t *in_tree = (uint8_t *)malloc((size_t)2 * N);
    int32_t *tlo = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *thi = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *tree = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *lptr = (int32_t *)malloc(sizeof(int32_t) * (N + 1));
    double *wgt = (double *)malloc(sizeof(double) * N);
    double *U = (double *)malloc(sizeof(double) * N);
    double *A = (double *)malloc(sizeof(double) * N);
    double *s = (double *)malloc(sizeof(double) * N);
    double *best = (double *)malloc(sizeof(double) * N);
    double *second = (double *)malloc(sizeof(double) * N);

    or_edge_keys(left, H, W, level, key);
    /* Kruskal's edge order: the colour weights (MST), or for the random
     * spanning tree (RT, Section 4.1) the given random ranks, so that sorting
     * the edges by (rank, id) is the random shuffle; the aggregation weights
     * stay the colour weights of eq. weight either way */
    for (int i = 0; i < 2 * N; ++i)
        order_key[i] = key[i] < 0 ? -1 : (rank ? rank[i] : key[i]);
    or_kruskal(H, W, order_key, pix_lo, pix_hi, beta_num, beta_den, in_tree,
               pix_lo ? tlo : NULL, pix_lo ? thi : NULL);
    if (!pix_lo)
        for (int v = 0; v < N; ++v) { tlo[v] = 0; thi[v] = dmax; }
    int nl = or_root_forest(H, W, in_tree, key, level, parent, wgt, depth, tree, order, lptr);
    for (int v = 0; v < N; ++v) {
        s[v] = parent[v] >= 0 ? exp(-wgt[v] / sigma) : 0.0;
        best[v] = INFINITY; second[v] = INFINITY; disp[v] = -1;
    }
    for (int x = 0; x <= dmax; ++x) {
        /* E(., x) on the trees whose interval holds x, zero elsewhere */
        for (int v = 0; v < N; ++v)
            U[v] = (x >= tlo[v] && x <= thi[v])
                       ? or_matching_cost(left, right, H, W, v % W, v / W, x, prm) : 0.0;
        for (int i = N - 1; i >= 0; --i) {
            int v = order[i];
            if (parent[v] >= 0) U[parent[v]] += s[v] * U[v];
        }
        for (int i = 0; i < N; ++i) {
            int v = order[i];
            A[v] = parent[v] < 0 ? U[v] : s[v] * A[parent[v]] + (1.0 - s[v] * s[v]) * U[v];
        }
        for (int v = 0; v < N; ++v) {
            if (x < tlo[v] || x > thi[v]) continue;
            if (A[v] < best[v]) { second[v] = best[v]; best[v] = A[v]; disp[v] = x; }
            else if (A[v] < second[v]) second[v] = A[v];
        }
        for (int k = 0; k < n_sample; ++k)
            if (sample_d[k] == x)
                for (int v = 0; v < N; ++v)
                    sample_agg[(size_t)k * N + v] = (x >= tlo[v] && x <= thi[v]) ? A[v] : NAN;
    }
    if (c1) memcpy(c1, best, sizeof(double) * N);
    if (c2) memcpy(c2, second, sizeof(double) * N);
    if (parent_o) memcpy(parent_o, parent, sizeof(int32_t) * N);
    if (depth_o) memcpy(depth_o, depth, sizeof(int32_t) * N);
    if (order_o) memcpy(order_o, order, sizeof(int32_t) * N);
    if (level_ptr_o) memcpy(level_ptr_o, lptr, sizeof(int32_t) * (nl + 1));
    if (tree_lo_o) memcpy(tree_lo_o, tlo, sizeof(int32_t) * N);
    if (tree_hi_o) memcpy(tree_hi_o, thi, sizeof(int32_t) * N);
    free(key); free(order_key); free(in_tree); free(tlo); free(thi); free(parent); free(depth);
    free(tree);
    free(order); free(lptr); free(wgt); free(U); free(A); free(s); free(best); free(second);
    return nl;
}

/* ------------------------------------------------------------------------ */
/* Gradients of L = sum_{i,x} g(i,x) * agg(i,x) with agg = A C,
 * A_ij = exp(-D(i,j)/sigma) on the forest (0 across trees).
 *
 * Plain definition (dense; tiny inputs only):
 *   dL/dC(j,x)  = sum_i g(i,x) A_ij
 *   dL/dsigma   = sum_{i,j,x} g(i,x) A_ij D(i,j)/sigma^2 C(j,x)
 *   dL/dw_e     = -(1/sigma) sum over pairs (i,j) whose path holds e of
 *                 sum_x g(i,x) A_ij C(j,x)
 * For each source i a traversal of its tree gives D(i,.) and, accumulated from
 * the leaves of that traversal, the pair sums that cross each edge.
 * dw is indexed by grid edge id (2N entries, 0 off the forest). */

OR_API void or_aggregate_grad_dense(int H, int W, const uint8_t *in_tree, const double *edge_w,
                                    double sigma, int D, const double *cost, const double *g,
                                    double *dC, double *dw, double *dsigma) {
    int N = H * W;
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *seq = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *from = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *fedge = (int32_t *)malloc(sizeof(int32_t) * N);
    double *plen = (double *)malloc(sizeof(double) * N);
    double *acc = (double *)malloc(sizeof(double) * N);
    for (size_t k = 0; k < (size_t)N * D; ++k) dC[k] = 0.0;
    for (int k = 0; k < 2 * N; ++k) dw[k] = 0.0;
    double ds = 0.0;
    for (int i = 0; i < N; ++i) {
        int sp = 0, ns = 0;
        stack[sp++] = i; from[i] = -1; fedge[i] = -1; plen[i] = 0.0;
        while (sp) {
            int v = stack[--sp];
            seq[ns++] = v;
            for (int k = 0; k < 4; ++k) {
                int q, id = nbr_edge(H, W, v, k, &q);
                if (id < 0 || !in_tree[id] || q == from[v]) continue;
                from[q] = v; fedge[q] = id; plen[q] = plen[v] + edge_w[id];
                stack[sp++] = q;
            }
        }
        const double *gi = g + (size_t)i * D;
        for (int t = 0; t < ns; ++t) {
            int j = seq[t];
            double a = exp(-plen[j] / sigma);
            const double *cj = cost + (size_t)j * D;
            double pair = 0.0;
            for (int x = 0; x < D; ++x) {
                dC[(size_t)j * D + x] += gi[x] * a;
                pair += gi[x] * a * cj[x];
            }
            ds += pair * plen[j] / (sigma * sigma);
            acc[j] = pair;
        }
        /* children appear after their parent in seq: fold from the end */
        for (int t = ns - 1; t > 0; --t) {
            int j = seq[t];
            dw[fedge[j]] += -acc[j] / sigma;
            acc[from[j]] += acc[j];
        }
    }
    *dsigma = ds;
    free(stack); free(seq); free(from); free(fedge); free(plen); free(acc);
}

/* Two-pass form of the same gradients on a rooted forest (parent/order as in
 * or_root_forest).  The operator is symmetric, so dL/dC = A g is the two-pass
 * aggregation of g.  For the edge e = (v, parent p), the pairs whose path
 * crosses e are (subtree of v) x (rest) and back, which gives
 *   dL/ds_e = sum_x [ U_g(v) (A_C(p) - s_e U_C(v)) + U_C(v) (A_g(p) - s_e U_g(v)) ]
 * with U, A the up and down sums of C and of g; s_e = exp(-w_e/sigma),
 *   dL/dw_e = -(s_e/sigma) dL/ds_e,   dL/dsigma = sum_e dL/ds_e s_e w_e / sigma^2.
 * dw is per node (edge to its parent; 0 at roots). */

OR_API void or_aggregate_backward_twopass(int N, const int32_t *parent, const double *wgt,
                                          const int32_t *order, double sigma, int D,
                                          const double *cost, const double *g,
                                          double *dC, double *dw, double *dsigma) {
    size_t ND = (size_t)N * D;
    double *UC = (double *)malloc(sizeof(double) * ND);
    double *AC = (double *)malloc(sizeof(double) * ND);
    double *Ug = (double *)malloc(sizeof(double) * ND);
    memcpy(UC, cost, sizeof(double) * ND);
    memcpy(Ug, g, sizeof(double) * ND);
    for (int i = N - 1; i >= 0; --i) {
        int v = order[i], p = parent[v];
        if (p < 0) continue;
        double s = exp(-wgt[v] / sigma);
        for (int x = 0; x < D; ++x) {
            UC[(size_t)p * D + x] += s * UC[(size_t)v * D + x];
            Ug[(size_t)p * D + x] += s * Ug[(size_t)v * D + x];
        }
    }
    for (int i = 0; i < N; ++i) {
        int v = order[i], p = parent[v];
        for (int x = 0; x < D; ++x) {
            size_t k = (size_t)v * D + x;
            if (p < 0) { AC[k] = UC[k]; dC[k] = Ug[k]; continue; }
            double s = exp(-wgt[v] / sigma);
            AC[k] = s * AC[(size_t)p * D + x] + (1.0 - s * s) * UC[k];
            dC[k] = s * dC[(size_t)p * D + x] + (1.0 - s * s) * Ug[k];
        }
    }
    double ds = 0.0;
    for (int v = 0; v < N; ++v) {
        int p = parent[v];
        if (p < 0) { dw[v] = 0.0; continue; }
        double s = exp(-wgt[v] / sigma), acc = 0.0;
        for (int x = 0; x < D; ++x) {
            size_t kv = (size_t)v * D + x, kp = (size_t)p * D + x;
            acc += Ug[kv] * (AC[kp] - s * UC[kv]) + UC[kv] * (dC[kp] - s * Ug[kv]);
        }
        dw[v] = -(s / sigma) * acc;
        ds += acc * s * wgt[v] / (sigma * sigma);
    }
    *dsigma = ds;
    free(UC); free(AC); free(Ug);
}
