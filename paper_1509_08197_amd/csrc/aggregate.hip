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
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace hdp {

constexpr int kRowsPerGroup = 8;

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

// Coefficient of row r: zero where a chain starts (scan order), so the value
// carried in from the previous row is dropped there.
template <bool UP>
__device__ __forceinline__ double row_coef(const PassArgs &A, int64_t r) {
    if (UP) return (r + 1 < A.r1 && A.heavy[r + 1]) ? A.s[r + 1] : 0.0;
    return A.heavy[r] ? A.s[r] : 0.0;
}

// Constant term of row r for column j.
template <bool UP>
__device__ __forceinline__ double row_b(const PassArgs &A, int64_t r, int j) {
    if (UP) {
        double x = (double)A.src[r * A.width + j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int c = A.lc[(int64_t)k * A.n + r];
            if (c >= 0) x += A.s[c] * (double)A.aux[(int64_t)c * A.width + j];
        }
        return x;
    }
    double x = A.om[r] * (double)A.src[r * A.width + j];
    int p = A.prow[r];
    if (!A.heavy[r] && p >= 0) x += A.s[r] * (double)A.aux[(int64_t)p * A.width + j];
    return x;
}

// Physical row of logical position li of tile t (logical order = scan order).
template <bool UP>
__device__ __forceinline__ int64_t tile_row(const PassArgs &A, int t, int li) {
    return UP ? (int64_t)A.r1 - 1 - ((int64_t)t * A.rows + li) : (int64_t)A.r0 + (int64_t)t * A.rows + li;
}

// Tile reduce: the affine map of the whole tile applied to 0 (X) and the
// product of its coefficients (P).  Only the rows after the tile's last chain
// start matter for X (the coefficient there is 0), so only those are read.
template <bool UP>
__global__ void __launch_bounds__(kBlock) k_tile_reduce(PassArgs A) {
    __shared__ double sP[kBlock];
    __shared__ double sX[kBlock];
    __shared__ int sZ[kBlock];
    int t = blockIdx.x;
    if (t >= A.ntiles) return;
    int tid = threadIdx.x;
    int g = tid / A.width, j = tid - g * A.width;
    bool active = g < A.groups;
    double av[kRowsPerGroup];
    double P = 1.0;
    int z = -1;
    if (active) {
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            int li = g * kRowsPerGroup + i;
            int64_t r = tile_row<UP>(A, t, li);
            bool in = UP ? r >= A.r0 : r < A.r1;
            double a = in ? row_coef<UP>(A, r) : 1.0;
            av[i] = a;
            P = a * P;
            if (a == 0.0) z = li;
        }
    }
    sZ[tid] = z;
    __syncthreads();
    int zt = -1;
    for (int q = 0; q < A.groups; ++q) {
        int zq = sZ[q * A.width];
        zt = zq > zt ? zq : zt;
    }
    double X = 0.0;
    if (active && g * kRowsPerGroup + kRowsPerGroup - 1 >= zt) {
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            int li = g * kRowsPerGroup + i;
            int64_t r = tile_row<UP>(A, t, li);
            bool in = UP ? r >= A.r0 : r < A.r1;
            if (in && li >= zt) X = av[i] * X + row_b<UP>(A, r, j);
        }
    }
    sP[tid] = P;
    sX[tid] = X;
    __syncthreads();
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
}

// Tile apply: outputs of the tile from its carry-in.
template <bool UP>
__global__ void __launch_bounds__(kBlock) k_tile_apply(PassArgs A) {
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
            if (in) {
                a = row_coef<UP>(A, r);
                b = row_b<UP>(A, r, j);
            }
            av[i] = a;
            bv[i] = b;
            X = a * X + b;
            P = a * P;
        }
    }
    sP[tid] = P;
    sX[tid] = X;
    __syncthreads();
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

// ---------------------------------------------------------------------------------
// Single-launch pass.  Tiles of all phases are taken in ticket order (phase by
// phase in scan order, tiles in scan order inside a phase).  A tile only waits
// for tiles with smaller tickets, which are already running, so the launch
// always drains:
//   - before reading rows of the previous phase (light children's U in the up
//     pass, parents' A in the down pass) it waits for that phase's completion
//     counter;
//   - its carry-in (a chain that crosses the tile boundary) comes from a
//     decoupled look-back over the preceding tiles' published maps.
// Every wait is bounded; on timeout an error word is set and the pass goes on
// (wrong values, never a hang).

struct PassPlan {
    int n_phases;
    int total_tiles;
    int32_t row0[HDP_MAX_PHASES + 1];   // rows of phase k: row0[k] .. row0[k+1]-1
    int32_t tile0[HDP_MAX_PHASES + 1];  // first ticket of the q-th processed phase
};

struct PassSync {
    int32_t *ticket;   // [1]
    int32_t *done;     // [HDP_MAX_PHASES] completed tiles per processed phase
    int32_t *flag;     // [tiles] 0 nothing, 1 map published, 2 final value published
    double *tP;        // [tiles] product of the tile's coefficients
    double *tX;        // [tiles][width] tile map applied to 0
    double *tI;        // [tiles][width] value after the tile's last row
    int32_t *err;      // nonzero: a bounded wait timed out
};

// Data that crosses workgroups inside one launch (published tile maps, rows of
// the previous phase, flags) is read and written with device-scope relaxed
// atomics (device-coherent loads/stores); a publisher waits for its stores to
// complete before it raises the flag.  No cache-wide flush or invalidate is
// issued.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_complete() { __builtin_amdgcn_s_waitcnt(0); }

constexpr int64_t kSpinLimit = int64_t(1) << 24;

// Bounded wait (one lane) until *p >= target.
__device__ void wait_at_least(const int32_t *p, int32_t target, int32_t *err, int code) {
    int64_t it = 0;
    while (ld_dev(p) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++it > kSpinLimit) {
            atomicMax(err, code);
            break;
        }
    }
}

__global__ void k_pass_init(PassSync sy, int total_tiles) {
    int64_t i = gtid();
    if (i < total_tiles) sy.flag[i] = 0;
    if (i < HDP_MAX_PHASES) sy.done[i] = 0;
    if (i == 0) sy.ticket[0] = 0;
}

template <bool UP>
__global__ void __launch_bounds__(kBlock) k_agg_pass(PassArgs A, PassPlan pl, PassSync sy) {
    __shared__ double sP[kBlock];
    __shared__ double sX[kBlock];
    __shared__ int s_ticket, s_flag;
    __shared__ double s_first;
    const int tid = threadIdx.x;
    if (tid == 0) s_ticket = atomicAdd(sy.ticket, 1);
    __syncthreads();
    const int T = s_ticket;
    if (T >= pl.total_tiles) return;
    int q = 0;
    while (q + 1 < pl.n_phases && pl.tile0[q + 1] <= T) ++q;
    const int k = UP ? pl.n_phases - 1 - q : q;
    const int tl = T - pl.tile0[q];
    A.r0 = pl.row0[k];
    A.r1 = pl.row0[k + 1];
    const int g = tid / A.width, j = tid - g * A.width;
    const bool active = g < A.groups;
    const int w = A.width;

    // stage 1: loads that do not depend on other tiles
    double av[kRowsPerGroup], bv[kRowsPerGroup];
    int32_t rr[kRowsPerGroup];
    int32_t x0[kRowsPerGroup], x1[kRowsPerGroup], x2[kRowsPerGroup];
    if (active) {
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            int li = g * kRowsPerGroup + i;
            int r = UP ? A.r1 - 1 - (tl * A.rows + li) : A.r0 + tl * A.rows + li;
            bool in = UP ? r >= A.r0 : r < A.r1;
            rr[i] = in ? r : -1;
            av[i] = 1.0;
            bv[i] = 0.0;
            x0[i] = x1[i] = x2[i] = -1;
            if (!in) continue;
            av[i] = row_coef<UP>(A, r);
            if (UP) {
                bv[i] = (double)A.src[r * w + j];
                x0[i] = A.lc[r];
                x1[i] = A.lc[(int)A.n + r];
                x2[i] = A.lc[2 * (int)A.n + r];
            } else {
                bv[i] = A.om[r] * (double)A.src[r * w + j];
                x0[i] = A.heavy[r] ? -1 : A.prow[r];
            }
        }
    }
    // the previous phase must be complete before its rows are read
    if (q > 0) {
        if (tid == 0) wait_at_least(&sy.done[q - 1], pl.tile0[q] - pl.tile0[q - 1], sy.err, 16);
        __syncthreads();
    }
    // stage 2: rows of the previous phase (light children / parent)
    double P = 1.0, X = 0.0;
    if (active) {
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            if (UP) {
                if (x0[i] >= 0) bv[i] += A.s[x0[i]] * (double)ld_dev(&A.aux[x0[i] * w + j]);
                if (x1[i] >= 0) bv[i] += A.s[x1[i]] * (double)ld_dev(&A.aux[x1[i] * w + j]);
                if (x2[i] >= 0) bv[i] += A.s[x2[i]] * (double)ld_dev(&A.aux[x2[i] * w + j]);
            } else if (x0[i] >= 0) {
                bv[i] += A.s[rr[i]] * (double)ld_dev(&A.aux[x0[i] * w + j]);
            }
            X = av[i] * X + bv[i];
            P = av[i] * P;
        }
    }
    if (tid == 0) s_first = av[0];
    sP[tid] = P;
    sX[tid] = X;
    __syncthreads();
    // map of the whole tile for column j (P is the same in every column)
    double Pt = 1.0, Xt = 0.0;
    if (active) {
        for (int q2 = 0; q2 < A.groups; ++q2) {
            double pq = sP[q2 * A.width + j];
            Xt = pq * Xt + sX[q2 * A.width + j];
            Pt = pq * Pt;
        }
    }
    const bool incl_now = tl == 0 || Pt == 0.0;
    if (active && g == 0) {
        if (incl_now) {
            st_dev(&sy.tI[T * w + j], Xt);
        } else {
            st_dev(&sy.tX[T * w + j], Xt);
            if (j == 0) st_dev(&sy.tP[T], Pt);
        }
    }
    stores_complete();
    __syncthreads();
    if (tid == 0) st_dev(&sy.flag[T], incl_now ? 2 : 1);

    // carry-in (decoupled look-back), needed when the first row continues a chain
    double carry = 0.0;
    if (tl > 0 && s_first != 0.0) {
        double mP = 1.0, mX = 0.0;
        int kk = T - 1;
        for (;;) {
            if (tid == 0) {
                int64_t it = 0;
                int f;
                while ((f = ld_dev(&sy.flag[kk])) == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++it > kSpinLimit) {
                        atomicMax(sy.err, 17);
                        f = 2;
                        break;
                    }
                }
                s_flag = f;
            }
            __syncthreads();
            int f = s_flag;
            if (f == 2) {
                if (active) carry = mP * ld_dev(&sy.tI[kk * w + j]) + mX;
                break;
            }
            if (active) {
                double pk = ld_dev(&sy.tP[kk]);
                mX = mP * ld_dev(&sy.tX[kk * w + j]) + mX;
                mP = mP * pk;
            }
            --kk;
            __syncthreads();
            if (kk < pl.tile0[q]) break;  // unreachable: a phase's first tile publishes its value
        }
    }

    // apply and store
    if (active) {
        double c = carry;
        for (int q2 = 0; q2 < g; ++q2) c = sP[q2 * A.width + j] * c + sX[q2 * A.width + j];
#pragma unroll
        for (int i = 0; i < kRowsPerGroup; ++i) {
            c = av[i] * c + bv[i];
            if (rr[i] >= 0) st_dev(&A.dst[rr[i] * w + j], (float)c);
        }
        if (!incl_now && g == A.groups - 1) st_dev(&sy.tI[T * w + j], c);
    }
    stores_complete();
    __syncthreads();
    if (tid == 0) {
        if (!incl_now) st_dev(&sy.flag[T], 2);
        atomicAdd(&sy.done[q], 1);
    }
}

// --- workspace --------------------------------------------------------------------

struct AggWs {
    int32_t *flag, *done, *ticket;
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
    a.flag = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * nt));
    a.done = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * HDP_MAX_PHASES));
    a.ticket = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 4));
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
    k_tile_reduce<UP><<<A.ntiles, kBlock, 0, st>>>(A);
    k_carry<<<A.width, kBlock, 0, st>>>(A);
    k_tile_apply<UP><<<A.ntiles, kBlock, 0, st>>>(A);
}

static int schedule_mode() {
    static int mode = -1;
    if (mode < 0) {
        const char *e = getenv("HDP_AGG_SCHEDULE");
        mode = (e && e[0] == '3') ? 3 : 1;  // 1: one launch per pass, 3: three launches per phase
    }
    return mode;
}

template <bool UP>
static void run_pass_single(PassArgs A, const int32_t *phase_ptr, int n_phases, const AggWs &w,
                            int32_t *err, hipStream_t st) {
    PassPlan pl{};
    pl.n_phases = n_phases;
    int tot = 0;
    for (int q = 0; q < n_phases; ++q) {
        int k = UP ? n_phases - 1 - q : q;
        int rows = phase_ptr[k + 1] - phase_ptr[k];
        pl.tile0[q] = tot;
        tot += (rows + A.rows - 1) / A.rows;
    }
    pl.tile0[n_phases] = tot;
    for (int k = 0; k <= n_phases; ++k) pl.row0[k] = phase_ptr[k];
    pl.total_tiles = tot;
    if (tot == 0) return;
    PassSync sy{w.ticket, w.done, w.flag, w.Pt, w.Xt, w.Ct, err};
    int64_t init_n = tot > HDP_MAX_PHASES ? tot : HDP_MAX_PHASES;
    k_pass_init<<<grid_for(init_n), kBlock, 0, st>>>(sy, tot);
    k_agg_pass<UP><<<tot, kBlock, 0, st>>>(A, pl, sy);
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
    if (schedule_mode() == 1) {
        A.src = src; A.aux = up; A.dst = up;
        run_pass_single<true>(A, phase_ptr, n_phases, w, f.info + HDP_INFO_ERROR, st);
        A.src = up; A.aux = out; A.dst = out;
        run_pass_single<false>(A, phase_ptr, n_phases, w, f.info + HDP_INFO_ERROR, st);
        return;
    }
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
        A.src = cost; A.aux = w.up; A.dst = w.up;
        if (schedule_mode() == 1) {
            run_pass_single<true>(A, phase_ptr, n_phases, w, f.info + HDP_INFO_ERROR, st);
        } else {
            for (int k = n_phases - 1; k >= 0; --k) {
                A.r0 = phase_ptr[k]; A.r1 = phase_ptr[k + 1];
                run_pass<true>(A, st);
            }
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
