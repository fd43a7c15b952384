// Tree aggregation (eq. W, eq. S, eq. C) and its adjoint.
//
// The aggregated cost agg(v,x) = sum_u exp(-W(v,u)/sigma) cost(u,x) is computed
// exactly by two passes over the forest (the linear-time scheme of the tree
// methods, Section 1):
//   up   U(v) = C(v) + sum_{children c} s_c U(c)            (leaves first)
//   down A(v) = s_v A(parent) + (1 - s_v^2) U(v), A(root) = U(root)
// with s_v = exp(-w(v,parent)/sigma).
//
// Schedule.  The forest's rows are grouped in chain phases (heavy-path
// decomposition, at most log2(n)+1 phases).  Along a heavy path both passes are
// first-order linear recurrences with a scalar coefficient per row,
//   up:   U_r = b_r + a_r U_{r+1},  a_r = s_{r+1} if row r+1 is r's heavy child
//         b_r = C_r + sum over light children c of s_c U_c (earlier phase)
//   down: A_r = a_r A_{r-1} + b_r,  a_r = s_r if r is a heavy child
//         b_r = (1 - s_r^2) U_r + (r heads a chain ? s_r A_parent : 0)
// and a zero coefficient ends a chain.  So each phase is ONE segmented scan of
// affine maps over a contiguous range of rows, independent per label column:
// tile reduce -> carry scan over tiles -> tile apply.  Rows are row-major
// [row][width] (labels fastest); arithmetic is FP64 in registers, storage FP32.
#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

constexpr int kRowsPerGroup = 16;

struct AggTileGeom {
    int width;   // labels per row (<= 256)
    int groups;  // row groups per tile = 256 / width
    int rows;    // rows per tile = groups * kRowsPerGroup
};

static AggTileGeom tile_geom(int width) {
    AggTileGeom t;
    t.width = width;
    t.groups = kBlock / width;
    if (t.groups < 1) t.groups = 1;
    t.rows = t.groups * kRowsPerGroup;
    return t;
}

__global__ void k_coef(int64_t n, const float *__restrict__ rw, const int32_t *__restrict__ prow,
                       double inv_sigma, double *__restrict__ s, double *__restrict__ om) {
    int64_t r = gtid();
    if (r >= n) return;
    if (prow[r] < 0) {
        s[r] = 0.0;
        om[r] = 1.0;
    } else {
        double w = (double)rw[r];
        s[r] = exp(-w * inv_sigma);
        om[r] = -expm1(-2.0 * w * inv_sigma);
    }
}

struct PassArgs {
    int64_t n;
    int32_t r0, r1;          // rows of the phase
    int width;
    int rows;                // rows per tile
    int groups;
    int ntiles;
    const double *s, *om;
    const uint8_t *heavy;
    const int32_t *prow;
    const int32_t *lc;       // [3][n]
    const float *src;        // up: cost C;  down: U
    const float *aux;        // up: U (light children, earlier phase);  down: A (parents)
    float *dst;              // up: U;  down: A
    double *Pt, *Xt, *Ct;    // per tile: coefficient product, zero-input result, carry-in
};

// Affine map of one row: x -> a x + b for column j.
template <bool UP>
__device__ __forceinline__ void row_map(const PassArgs &A, int64_t r, int j, double &a, double &b) {
    if (UP) {
        a = (r + 1 < A.r1 && A.heavy[r + 1]) ? A.s[r + 1] : 0.0;
        double x = (double)A.src[r * A.width + j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int c = A.lc[(int64_t)k * A.n + r];
            if (c >= 0) x += A.s[c] * (double)A.aux[(int64_t)c * A.width + j];
        }
        b = x;
    } else {
        bool hv = A.heavy[r];
        double s = A.s[r];
        a = hv ? s : 0.0;
        double x = A.om[r] * (double)A.src[r * A.width + j];
        int p = A.prow[r];
        if (!hv && p >= 0) x += s * (double)A.aux[(int64_t)p * A.width + j];
        b = x;
    }
}

// Physical row of logical position li of tile t (logical order = scan order).
template <bool UP>
__device__ __forceinline__ int64_t tile_row(const PassArgs &A, int t, int li) {
    return UP ? (int64_t)A.r1 - 1 - ((int64_t)t * A.rows + li) : (int64_t)A.r0 + (int64_t)t * A.rows + li;
}

// APPLY = false: per-tile (P, X) with zero input.  APPLY = true: outputs from
// the tile's carry-in.
template <bool UP, bool APPLY>
__global__ void __launch_bounds__(kBlock) k_tile(PassArgs A) {
    __shared__ double sP[kBlock];
    __shared__ double sX[kBlock];
    int t = blockIdx.x;
    if (t >= A.ntiles) return;
    int tid = threadIdx.x;
    int g = tid / A.width, j = tid - g * A.width;
    bool active = g < A.groups;
    double av[kRowsPerGroup], bv[kRowsPerGroup];
    int64_t rr[kRowsPerGroup];
    double P = 1.0, X = 0.0;
    if (active) {
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            int li = g * kRowsPerGroup + i;
            int64_t r = tile_row<UP>(A, t, li);
            bool in = UP ? r >= A.r0 : r < A.r1;
            rr[i] = in ? r : -1;
            double a = 1.0, b = 0.0;  // identity map past the end of the phase
            if (in) row_map<UP>(A, r, j, a, b);
            av[i] = a;
            bv[i] = b;
            X = a * X + b;
            P = a * P;
        }
    }
    sP[tid] = P;
    sX[tid] = X;
    __syncthreads();
    if (!APPLY) {
        if (active && g == 0) {
            double Pc = 1.0, Xc = 0.0;
            for (int q = 0; q < A.groups; ++q) {
                double pq = sP[q * A.width + j], xq = sX[q * A.width + j];
                Xc = pq * Xc + xq;
                Pc = pq * Pc;
            }
            A.Xt[(int64_t)t * A.width + j] = Xc;
            if (j == 0) A.Pt[t] = Pc;
        }
        return;
    }
    if (!active) return;
    double c = A.Ct[(int64_t)t * A.width + j];
    for (int q = 0; q < g; ++q) c = sP[q * A.width + j] * c + sX[q * A.width + j];
#pragma unroll
    for (int i = 0; i < kRowsPerGroup; ++i) {
        c = av[i] * c + bv[i];
        if (rr[i] >= 0) A.dst[rr[i] * A.width + j] = (float)c;
    }
}

// Carry-in of every tile, one workgroup per label column: exclusive scan of
// the tiles' affine maps (composition in scan order), starting from 0.
__global__ void __launch_bounds__(kBlock) k_carry(PassArgs A) {
    __shared__ double sP[kBlock];
    __shared__ double sX[kBlock];
    int j = blockIdx.x;
    int tid = threadIdx.x;
    int chunk = (A.ntiles + kBlock - 1) / kBlock;
    int t0 = tid * chunk, t1 = t0 + chunk < A.ntiles ? t0 + chunk : A.ntiles;
    double P = 1.0, X = 0.0;
    for (int t = t0; t < t1; ++t) {
        double p = A.Pt[t];
        X = p * X + A.Xt[(int64_t)t * A.width + j];
        P = p * P;
    }
    sP[tid] = P;
    sX[tid] = X;
    __syncthreads();
    // inclusive Hillis-Steele scan of maps: combine(earlier e, later l) = (l.P e.P, l.P e.X + l.X)
    for (int off = 1; off < kBlock; off <<= 1) {
        double pe = 1.0, xe = 0.0;
        if (tid >= off) { pe = sP[tid - off]; xe = sX[tid - off]; }
        __syncthreads();
        if (tid >= off) {
            double pl = sP[tid], xl = sX[tid];
            sP[tid] = pl * pe;
            sX[tid] = pl * xe + xl;
        }
        __syncthreads();
    }
    double c = tid > 0 ? sX[tid - 1] : 0.0;
    for (int t = t0; t < t1; ++t) {
        A.Ct[(int64_t)t * A.width + j] = c;
        c = A.Pt[t] * c + A.Xt[(int64_t)t * A.width + j];
    }
}

// --- workspace --------------------------------------------------------------------

struct AggWs {
    double *s, *om, *Pt, *Xt, *Ct;
    float *up;      // U when the caller does not keep it
    float *ug;      // U of the gradient (backward)
    double *red;    // per-block partial sums (backward)
};

static int64_t max_tiles(int64_t n, int width) {
    AggTileGeom tg = tile_geom(width);
    return n / tg.rows + HDP_MAX_PHASES + 2;
}

static AggWs carve_agg_ws(void *ws, int64_t n, int width, size_t *bytes) {
    char *base = reinterpret_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t sz) {
        off = (off + 255) & ~size_t(255);
        char *p = base + off;
        off += sz < 1 ? 1 : sz;
        return p;
    };
    int64_t nt = max_tiles(n, width);
    AggWs a;
    a.s = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.om = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.Pt = reinterpret_cast<double *>(take(sizeof(double) * nt));
    a.Xt = reinterpret_cast<double *>(take(sizeof(double) * nt * width));
    a.Ct = reinterpret_cast<double *>(take(sizeof(double) * nt * width));
    a.up = reinterpret_cast<float *>(take(sizeof(float) * n * width));
    a.ug = reinterpret_cast<float *>(take(sizeof(float) * n * width));
    a.red = reinterpret_cast<double *>(take(sizeof(double) * (n / 4 + 64)));
    *bytes = off + 256;
    return a;
}

size_t aggregate_workspace_bytes(int64_t n, int width) {
    size_t b = 0;
    carve_agg_ws(nullptr, n, width, &b);
    return b;
}

template <bool UP>
static void run_pass(PassArgs A, hipStream_t st) {
    if (A.r1 <= A.r0) return;
    A.ntiles = (int)(((int64_t)A.r1 - A.r0 + A.rows - 1) / A.rows);
    k_tile<UP, false><<<A.ntiles, kBlock, 0, st>>>(A);
    k_carry<<<A.width, kBlock, 0, st>>>(A);
    k_tile<UP, true><<<A.ntiles, kBlock, 0, st>>>(A);
}

// Two passes of `src` over the forest: U -> up, A -> out.
static void two_pass(const hdp_forest &f, int width, const int32_t *phase_ptr, int n_phases,
                     const float *src, float *up, float *out, const AggWs &w, hipStream_t st) {
    AggTileGeom tg = tile_geom(width);
    PassArgs A{};
    A.n = f.n;
    A.width = width;
    A.rows = tg.rows;
    A.groups = tg.groups;
    A.s = w.s;
    A.om = w.om;
    A.heavy = f.heavy;
    A.prow = f.prow;
    A.lc = f.lc;
    A.Pt = w.Pt;
    A.Xt = w.Xt;
    A.Ct = w.Ct;
    for (int k = n_phases - 1; k >= 0; --k) {
        A.r0 = phase_ptr[k];
        A.r1 = phase_ptr[k + 1];
        A.src = src;
        A.aux = up;
        A.dst = up;
        run_pass<true>(A, st);
    }
    for (int k = 0; k < n_phases; ++k) {
        A.r0 = phase_ptr[k];
        A.r1 = phase_ptr[k + 1];
        A.src = up;
        A.aux = out;
        A.dst = out;
        run_pass<false>(A, st);
    }
}

void launch_aggregate(const hdp_forest &f, int width, const int32_t *phase_ptr, int n_phases,
                      const float *cost, float sigma, float *agg, float *up, void *ws,
                      hipStream_t st) {
    size_t bytes;
    AggWs w = carve_agg_ws(ws, f.n, width, &bytes);
    k_coef<<<grid_for(f.n), kBlock, 0, st>>>(f.n, f.rw, f.prow, 1.0 / (double)sigma, w.s, w.om);
    two_pass(f, width, phase_ptr, n_phases, cost, up ? up : w.up, agg, w, st);
}

// --- adjoint ----------------------------------------------------------------------------

// Per row (edge to the parent): acc = sum_x [Ug (Ac(p) - s Uc) + Uc (Ag(p) - s Ug)];
// grad_w = -(s/sigma) acc; per-block partial of acc * s * w / sigma^2.
__global__ void __launch_bounds__(kBlock) k_edge_grad(int64_t n, int width,
                                                      const int32_t *__restrict__ prow,
                                                      const int32_t *__restrict__ node,
                                                      const float *__restrict__ rw,
                                                      const double *__restrict__ s,
                                                      const float *__restrict__ uc,
                                                      const float *__restrict__ ac,
                                                      const float *__restrict__ ug,
                                                      const float *__restrict__ ag, double inv_sigma,
                                                      float *__restrict__ grad_w,
                                                      double *__restrict__ red) {
    __shared__ double part[kBlock / 64];
    int64_t r = gtid() >> 6;
    int lane = threadIdx.x & 63;
    double contrib = 0.0;
    if (r < n) {
        int p = prow[r];
        double acc = 0.0;
        double sr = s[r];
        if (p >= 0) {
            const float *ucr = uc + r * width, *ugr = ug + r * width;
            const float *acp = ac + (int64_t)p * width, *agp = ag + (int64_t)p * width;
            for (int j = lane; j < width; j += 64) {
                double u1 = ucr[j], u2 = ugr[j];
                acc += u2 * ((double)acp[j] - sr * u1) + u1 * ((double)agp[j] - sr * u2);
            }
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0 && grad_w) grad_w[node[r]] = p >= 0 ? (float)(-(sr * inv_sigma) * acc) : 0.f;
        if (p >= 0) contrib = acc * sr * (double)rw[r] * inv_sigma * inv_sigma;
    }
    if (lane == 0) part[threadIdx.x >> 6] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += part[k];
        red[blockIdx.x] = t;
    }
}

__global__ void k_sum_red(const double *__restrict__ red, int64_t nb, float *__restrict__ out) {
    __shared__ double sh[kBlock];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += kBlock) t += red[i];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)sh[0];
}

void launch_aggregate_backward(const hdp_forest &f, int width, const int32_t *phase_ptr,
                               int n_phases, const float *cost, const float *agg, const float *up,
                               const float *grad_agg, float sigma, float *grad_cost, float *grad_w,
                               float *grad_sigma, void *ws, hipStream_t st) {
    size_t bytes;
    AggWs w = carve_agg_ws(ws, f.n, width, &bytes);
    k_coef<<<grid_for(f.n), kBlock, 0, st>>>(f.n, f.rw, f.prow, 1.0 / (double)sigma, w.s, w.om);
    const float *uc = up;
    if (!uc) {  // recompute the up pass of the cost (the down pass output is discarded)
        AggTileGeom tg = tile_geom(width);
        PassArgs A{};
        A.n = f.n; A.width = width; A.rows = tg.rows; A.groups = tg.groups;
        A.s = w.s; A.om = w.om; A.heavy = f.heavy; A.prow = f.prow; A.lc = f.lc;
        A.Pt = w.Pt; A.Xt = w.Xt; A.Ct = w.Ct;
        for (int k = n_phases - 1; k >= 0; --k) {
            A.r0 = phase_ptr[k]; A.r1 = phase_ptr[k + 1];
            A.src = cost; A.aux = w.up; A.dst = w.up;
            run_pass<true>(A, st);
        }
        uc = w.up;
    }
    two_pass(f, width, phase_ptr, n_phases, grad_agg, w.ug, grad_cost, w, st);
    if (grad_w || grad_sigma) {
        int64_t nb = (f.n * 64 + kBlock - 1) / kBlock;
        k_edge_grad<<<(unsigned)nb, kBlock, 0, st>>>(f.n, width, f.prow, f.node, f.rw, w.s, uc, agg,
                                                    w.ug, grad_cost, 1.0 / (double)sigma, grad_w,
                                                    w.red);
        if (grad_sigma) k_sum_red<<<1, kBlock, 0, st>>>(w.red, nb, grad_sigma);
    }
}

}  // namespace hdp
