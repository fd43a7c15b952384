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
//         b_r = C_r + sum over light children c of s_c U_c (previous phase)
//   down: A_r = a_r A_{r-1} + b_r,  a_r = s_r if r is a heavy child
//         b_r = (1 - s_r^2) U_r + (r heads a chain ? s_r A_parent : 0)
// and a zero coefficient ends a chain.  Each pass is ONE launch: tiles of
// consecutive rows are taken in ticket order (phase by phase in scan order),
// a tile waits only for the tiles that produced the previous-phase rows it
// reads, and the carry of a chain that crosses tile boundaries comes from a
// decoupled look-back over the preceding tiles' affine maps (64 tiles per
// step).  Rows are row-major [row][width] (labels fastest); arithmetic is FP64
// in registers, storage FP32.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"
#include "matchcost.hpp"

namespace hdp {

constexpr int kRPGDefault = 8;  // rows per thread group of a tile
constexpr int kSumBlocks = 512;  // blocks of the first summing launch of the adjoint

// Narrow rows use rows as signals: unwritten values hold signalling-NaN
// patterns that no arithmetic produces.  Rows of at most 64 labels, and rows
// of up to kSentMaxWidth labels that split into four labels per thread, are
// narrow; the others take the wide-row kernel with tile flags.
constexpr int kSentMaxWidth = 256;
__host__ __device__ inline bool narrow_rows(int width) {
    return width <= 64 || (width <= kSentMaxWidth && width % 4 == 0);
}
constexpr uint32_t kSentF = 0x7fa00001u;
constexpr uint64_t kSent64 = 0x7fa000017fa00001ull;
constexpr uint64_t kSentD = 0x7ff4000000000001ull;
// A narrow-row tile is one workgroup of kNarrowThreads threads; its map is
// scanned in kNarrowSegs segments of thread groups.  (512-thread tiles, half
// the tickets per row, measured slower on batches: the longer in-tile scan
// costs more than the ticket counter saves.)
constexpr int kNarrowThreads = 256;
constexpr int kNarrowSegs = kNarrowThreads / 64;


// Layout of the device-side pass plan (int32 words).
enum {
    P_NPH = 0,      // number of phases K
    P_TOT_UP = 1,   // tiles of the up pass
    P_TOT_DN = 2,   // tiles of the down pass
    P_ROWS = 3,     // rows per tile
    P_ROW0 = 4,     // [K+1] first row of phase k
    P_T0UP = 48,    // [K+1] first ticket of the q-th phase processed by the up pass
    P_T0DN = 96,    // [K+1] same for the down pass
    P_WORDS = 144
};

struct TileGeom {
    int cpt;     // labels per thread (4, 2 or 1)
    int rpg;     // rows per thread group (4, 8 or 16)
    int lpr;     // threads per row
    int groups;  // row groups per tile
    int rows;    // rows per tile
};

// Schedule chosen per row width (0 = built-in default), set by the tuner.
static int g_sched_cpt[HDP_MAX_LABELS + 1];
static int g_sched_rpg[HDP_MAX_LABELS + 1];

static bool schedule_valid(int width, int cpt, int rpg) {
    if (cpt != 1 && cpt != 2 && cpt != 4) return false;
    if (rpg != 4 && rpg != 8 && rpg != 16) return false;
    if (width % cpt != 0) return false;
    if (rpg == 16 && cpt != 2) return false;  // register budget
    return true;
}

static TileGeom make_geom(int width, int cpt, int rpg) {
    TileGeom t;
    t.cpt = cpt;
    t.rpg = rpg;
    t.lpr = (width + cpt - 1) / cpt;
    t.groups = (narrow_rows(width) ? kNarrowThreads : kBlock) / t.lpr;
    if (t.groups < 1) t.groups = 1;
    t.rows = t.groups * rpg;
    return t;
}

static TileGeom tile_geom(int width) {
    int cpt = g_sched_cpt[width], rpg = g_sched_rpg[width];
    if (!cpt || !schedule_valid(width, cpt, rpg)) {
        cpt = (width >= 48 && width % 4 == 0) ? 4 : (width % 2 == 0 && width >= 8) ? 2 : 1;
        // narrow rows: shorter tiles measured faster, except rows of 128 labels
        // or more (four labels per thread), where eight rows per group halve the
        // tiles: full-range step 4.40 -> 3.83 ms, 128-label adjoint 6.22 -> 5.88 ms
        rpg = narrow_rows(width) ? (width >= 128 && cpt == 4 ? 8 : 4) : kRPGDefault;
    }
    return make_geom(width, cpt, rpg);
}

bool set_schedule(int width, int cpt, int rpg) {
    if (width < 1 || width > HDP_MAX_LABELS) return false;
    if (cpt == 0) {
        g_sched_cpt[width] = g_sched_rpg[width] = 0;
        return true;
    }
    if (!schedule_valid(width, cpt, rpg)) return false;
    g_sched_cpt[width] = cpt;
    g_sched_rpg[width] = rpg;
    return true;
}

constexpr int kPassSets = 3;  // flag sets: up, down (and a second up pass in the adjoint)

// Prologue of an aggregation call, one launch: per-row coefficients
// s = exp(-w / sigma) and 1 - s^2, cleared tile flags and tickets of every
// pass, and (block 0) the ticket layout of both passes from the phase table.
__global__ void k_prologue(int64_t n, const float *__restrict__ rw,
                           const int32_t *__restrict__ prow, const uint8_t *__restrict__ heavy,
                           double inv_sigma, double *__restrict__ s, double *__restrict__ om,
                           int32_t *__restrict__ flags, int64_t tiles, int32_t *__restrict__ ticket,
                           const int32_t *__restrict__ phase_ptr, const int32_t *__restrict__ info,
                           int rows, int32_t *__restrict__ plan, uint32_t *__restrict__ fill0,
                           uint32_t *__restrict__ fill1, int width,
                           uint64_t *__restrict__ maps, int64_t map_words,
                           const float4 *__restrict__ imR, uint2 *__restrict__ imRp,
                           float rscale) {
    __shared__ int32_t sph[HDP_MAX_PHASES + 1];
    // One thread per row (the grid covers the rows and the tiles).
    const int64_t t = gtid();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // The phase table and the row's links and weight are loaded together,
    // before any of them is used (a thread past the last row reads the last
    // row and drops it).
    const int64_t rc = t < n ? t : n - 1;
    const int tx = (int)threadIdx.x;
    const int32_t ph = phase_ptr[tx <= HDP_MAX_PHASES ? tx : HDP_MAX_PHASES];
    int K = info[HDP_INFO_N_PHASES];
    const int pr = prow[rc];
    const uint8_t hv = heavy[rc];
    const float wf = rw[rc];
    // fused matching: the right image packed for the up pass (one pixel per
    // row: a layer has as many pixels as rows)
    const float4 rpx = imRp ? imR[rc] : make_float4(0.f, 0.f, 0.f, 0.f);
    K = K < 1 ? 1 : (K > HDP_MAX_PHASES ? HDP_MAX_PHASES : K);
    if (tx <= HDP_MAX_PHASES) sph[tx] = ph;
    __syncthreads();
    // Narrow rows: mark unwritten the rows of the up passes' outputs that a
    // tile polls (chain heads below a light edge, read by their parent's
    // tile, and the last row of every up-pass tile, read for the next tile's
    // carry).  The 64 rows of a wavefront are consecutive: the wavefront
    // stores the words of its marked rows together, lane j taking words
    // j, j + 64, ... of the block, so each store covers consecutive words.
    if (fill0 || fill1) {
        bool mark = false;
        if (t < n) {
            int lo = 0, hi = K - 1;  // phase of row t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sph[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const bool last = (sph[lo + 1] - (int)t) % rows == 0;
            mark = last || (pr >= 0 && !hv);
        }
        const uint64_t mm = __ballot(mark);
        const int lane = tx & 63;
        const int64_t r0w = t - lane;  // first row of the wavefront's block
        const bool even = (width & 1) == 0;
        const int hw = even ? width / 2 : width;  // words per row
        for (int idx = lane; idx < 64 * hw; idx += 64) {
            const int j = idx / hw;
            if (!((mm >> j) & 1ull)) continue;
            if (even) {
                const int64_t i = r0w * hw + idx;
                if (fill0) reinterpret_cast<uint64_t *>(fill0)[i] = kSent64;
                if (fill1) reinterpret_cast<uint64_t *>(fill1)[i] = kSent64;
            } else {
                const int64_t i = r0w * width + idx;
                if (fill0) fill0[i] = kSentF;
                if (fill1) fill1[i] = kSentF;
            }
        }
    }
    if (imRp && t < n) imRp[t] = pack_right(rpx, rscale);
    if (t < n) {
        if (pr < 0) {
            s[t] = 0.0;
            om[t] = 1.0;
        } else {
            const double w = (double)wf;
            s[t] = exp(-w * inv_sigma);
            om[t] = -expm1(-2.0 * w * inv_sigma);
        }
    }
    // the tile maps, marked unpublished
    for (int64_t i = t; i < map_words; i += stride) maps[i] = kSentD;
    if (t < tiles && !narrow_rows(width)) {  // tile flags: wide rows only (narrow rows signal by rows)
#pragma unroll
        for (int k = 0; k < 2 * kPassSets; ++k) flags[k * tiles + t] = 0;
    }
    if (t < kPassSets) ticket[t] = 0;
    if (t != 0) return;
    plan[P_NPH] = K;
    plan[P_ROWS] = rows;
    for (int k = 0; k <= K; ++k) plan[P_ROW0 + k] = phase_ptr[k];
    int tu = 0, td = 0;
    for (int q = 0; q < K; ++q) {
        int ku = K - 1 - q;
        plan[P_T0UP + q] = tu;
        tu += (phase_ptr[ku + 1] - phase_ptr[ku] + rows - 1) / rows;
        plan[P_T0DN + q] = td;
        td += (phase_ptr[q + 1] - phase_ptr[q] + rows - 1) / rows;
    }
    plan[P_T0UP + K] = tu;
    plan[P_T0DN + K] = td;
    plan[P_TOT_UP] = tu;
    plan[P_TOT_DN] = td;
}

struct PassArgs {
    int n;
    int width, lpr, groups, rows;
    const double *s, *om;
    const uint8_t *heavy;
    const int32_t *prow, *lc;
    const float *src;    // up: cost C;  down: U
    float *dst;          // up: U;  down: A  (rows of the previous phase are read back from it)
    const int32_t *plan;
    int32_t *ticket;     // [1]
    int32_t *flag;       // [tiles] 0 nothing, 1 map published, 2 final value published
    int32_t *flagw;      // [tiles] 1 once the tile's rows are stored
    double *tP;          // [tiles] product of the tile's coefficients
    double *tX;          // [tiles][width] tile map applied to 0
    double *tI;          // [tiles][width] value after the tile's last row
    int32_t *err;        // nonzero: a bounded wait timed out / inconsistent input
    // narrow-row mode (rows as signals)
    float *fill;         // up pass: rows of the following down pass's output to mark unwritten
    double *tPs, *tXs;   // this pass's tile maps (tiles without a chain break); tPs marked unwritten
    // fused matching (narrow rows): the up pass computes its cost rows from the
    // level images, the down pass writes each row's winning label
    const float4 *imL, *imR;
    const uint2 *imRp;  // right image packed by the prologue (8 bytes a pixel)
    float rinv;         // 4^-l: scale of the packed pixels
    CostParams cp;
    const int32_t *node, *rx, *rlh;
    int32_t *disp;
};

// Data that crosses workgroups inside one launch (published tile maps, rows of
// the previous phase, flags) is read and written with device-scope relaxed
// atomics (device-coherent loads and stores); a publisher waits for its stores
// to complete before it raises a flag.  No cache-wide flush or invalidate is
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
// ld_dev of element idx of an array of less than 4 GiB (32-bit byte offset)
template <typename T>
__device__ __forceinline__ T ld_dev32(const T *base, uint32_t idx) {
    return ld_dev(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                              (uint64_t)(idx * (uint32_t)sizeof(T))));
}

constexpr int kSpinLimit = 1 << 20;

__device__ __forceinline__ int wait_nonzero(const int32_t *p, int32_t *err, int code) {
    int f = ld_dev(p);
    int it = 0;
    while (f == 0) {
        __builtin_amdgcn_s_sleep(1);
        f = ld_dev(p);
        if (++it > kSpinLimit) {
            atomicMax(err, code);
            return 2;
        }
    }
    return f;
}

// CPT consecutive labels of one row: plain vector load (data of an earlier launch).
template <int CPT>
__device__ __forceinline__ void load_cols(const float *p, float *v) {
    if (CPT == 4) {
        float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else if (CPT == 2) {
        float2 x = *reinterpret_cast<const float2 *>(p);
        v[0] = x.x; v[1] = x.y;
    } else {
        v[0] = *p;
    }
}

// Device-coherent load / store of CPT consecutive labels (64-bit words).
template <int CPT>
__device__ __forceinline__ void load_cols_dev(const float *p, float *v) {
    if (CPT == 1) {
        v[0] = ld_dev(p);
    } else {
#pragma unroll
        for (int h = 0; h < CPT / 2; ++h) {
            uint64_t u = ld_dev(reinterpret_cast<const uint64_t *>(p) + h);
            v[2 * h] = __uint_as_float((uint32_t)u);
            v[2 * h + 1] = __uint_as_float((uint32_t)(u >> 32));
        }
    }
}

template <int CPT>
__device__ __forceinline__ void store_cols_dev(float *p, const double *c) {
    if (CPT == 1) {
        st_dev(p, (float)c[0]);
    } else {
#pragma unroll
        for (int h = 0; h < CPT / 2; ++h) {
            uint64_t u = (uint64_t)__float_as_uint((float)c[2 * h]) |
                         ((uint64_t)__float_as_uint((float)c[2 * h + 1]) << 32);
            st_dev(reinterpret_cast<uint64_t *>(p) + h, u);
        }
    }
}

template <bool UP, int CPT, int kRPG>
__global__ void __launch_bounds__(kBlock) k_pass(PassArgs A) {
    __shared__ double sP[kBlock];
    __shared__ double sX[kBlock * CPT];
    __shared__ int s_ticket;
    __shared__ int s_win[64];
    __shared__ double s_first;
    __shared__ int32_t s_plan[P_WORDS];
    const int tid = threadIdx.x;
    // the ticket, and meanwhile the whole plan into LDS (one word per thread)
    if (tid == 0) s_ticket = atomicAdd(A.ticket, 1);
    if (tid < P_WORDS) s_plan[tid] = A.plan[tid];
    __syncthreads();
    const int T = s_ticket;
    const int K = s_plan[P_NPH];
    const int total = s_plan[UP ? P_TOT_UP : P_TOT_DN];
    if (T >= total) return;
    const int32_t *t0 = s_plan + (UP ? P_T0UP : P_T0DN);
    const int32_t *row0 = s_plan + P_ROW0;
    int q = 0;
    while (q + 1 < K && t0[q + 1] <= T) ++q;
    const int k = UP ? K - 1 - q : q;
    const int tl = T - t0[q];
    const int r0 = row0[k], r1 = row0[k + 1];
    // the previous processed phase produced the rows gathered below
    const int kp = UP ? k + 1 : k - 1;
    const int pr0 = q > 0 ? row0[kp] : 0, pr1 = q > 0 ? row0[kp + 1] : 0;
    const int pt0 = q > 0 ? t0[q - 1] : 0, pt1 = t0[q];
    const int w = A.width, rows = A.rows;
    const int g = tid / A.lpr, jl = tid - g * A.lpr;
    const int j0 = jl * CPT;
    const bool active = g < A.groups;

    // stage 1: loads that do not depend on other tiles of this launch.  Row
    // maps x -> av * x + bv; the constant terms are sums of non-negative terms
    // held in FP32 (one relative rounding of at most 2^-24 per term added),
    // the maps are composed in FP64.
    double av[kRPG];
    float bv[kRPG][CPT];
    // row i of this thread's group (-1 past the phase), recomputed where used
    auto row_of = [&](int i) {
        const int li = g * kRPG + i;
        const int r = UP ? r1 - 1 - (tl * rows + li) : r0 + tl * rows + li;
        return active && (UP ? r >= r0 : r < r1) ? r : -1;
    };
    int x0[kRPG], x1[kRPG];
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
        const int r = row_of(i);
        const bool in = r >= 0;
        av[i] = 1.0;
        x0[i] = x1[i] = -1;
#pragma unroll
        for (int c = 0; c < CPT; ++c) bv[i][c] = 0.f;
        if (!in) continue;
        float v[CPT];
        load_cols<CPT>(A.src + (int64_t)r * w + j0, v);
        if (UP) {
            // heavy flag and coefficient of the next row, loaded together
            const int rn = r + 1 < r1 ? r + 1 : r;
            const bool hn = at32(A.heavy, rn);
            const double sn = at32(A.s, rn);
            av[i] = (r + 1 < r1 && hn) ? sn : 0.0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) bv[i][c] = v[c];
            x0[i] = at32(A.lc, r);
            x1[i] = at32(A.lc, A.n + r);
        } else {
            // heavy flag, coefficients and parent row, loaded together
            const bool hv = at32(A.heavy, r);
            const double sr = at32(A.s, r), o = at32(A.om, r);
            const int pr = at32(A.prow, r);
            av[i] = hv ? sr : 0.0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) bv[i][c] = (float)(o * (double)v[c]);
            x0[i] = hv ? -1 : pr;
        }
    }

    // stage 2: wait for the producing tiles of the gathered rows, then gather
    auto wait_row = [&](int x) {
        if (x < 0) return;
        if (x < pr0 || x >= pr1) {  // not in the previous phase: inconsistent forest
            atomicMax(A.err, 18);
            return;
        }
        int tk = pt0 + (UP ? (pr1 - 1 - x) / rows : (x - pr0) / rows);
        if (tk >= pt0 && tk < pt1) wait_nonzero(&A.flagw[tk], A.err, 16);
    };
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
        wait_row(x0[i]);
        if (UP) wait_row(x1[i]);
    }
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
        float v[CPT];
        if (UP) {
            if (x0[i] >= 0) {
                double sc = at32(A.s, x0[i]);
                load_cols_dev<CPT>(A.dst + (int64_t)x0[i] * w + j0, v);
#pragma unroll
                for (int c = 0; c < CPT; ++c) bv[i][c] = (float)((double)bv[i][c] + sc * (double)v[c]);
            }
            if (x1[i] >= 0) {
                double sc = at32(A.s, x1[i]);
                load_cols_dev<CPT>(A.dst + (int64_t)x1[i] * w + j0, v);
#pragma unroll
                for (int c = 0; c < CPT; ++c) bv[i][c] = (float)((double)bv[i][c] + sc * (double)v[c]);
            }
        } else if (x0[i] >= 0) {
            double sc = at32(A.s, row_of(i));
            load_cols_dev<CPT>(A.dst + (int64_t)x0[i] * w + j0, v);
#pragma unroll
            for (int c = 0; c < CPT; ++c) bv[i][c] = (float)((double)bv[i][c] + sc * (double)v[c]);
        }
    }

    // map of this thread's rows, then of the whole tile
    double P = 1.0, X[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) X[c] = 0.0;
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) X[c] = av[i] * X[c] + bv[i][c];
        P *= av[i];
    }
    if (tid == 0) s_first = av[0];
    sP[tid] = P;
#pragma unroll
    for (int c = 0; c < CPT; ++c) sX[tid * CPT + c] = X[c];
    __syncthreads();
    double Pt = 1.0, Xt[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) Xt[c] = 0.0;
    if (active) {
#pragma unroll 1
        for (int q2 = 0; q2 < A.groups; ++q2) {
            int o = q2 * A.lpr + jl;
            double pq = sP[o];
#pragma unroll
            for (int c = 0; c < CPT; ++c) Xt[c] = pq * Xt[c] + sX[o * CPT + c];
            Pt *= pq;
        }
    }
    const bool incl_now = tl == 0 || Pt == 0.0;
    if (active && g == 0) {
        double *dstp = incl_now ? A.tI : A.tX;
#pragma unroll
        for (int c = 0; c < CPT; ++c) st_dev(&dstp[(int64_t)T * w + j0 + c], Xt[c]);
        if (!incl_now && jl == 0) st_dev(&A.tP[T], Pt);
    }
    stores_complete();
    __syncthreads();
    if (tid == 0) st_dev(&A.flag[T], incl_now ? 2 : 1);

    // Carry-in by decoupled look-back, 64 predecessors per step: the nearest
    // tile that published its value, then the maps of the tiles after it
    // applied forward one tile at a time.  A tile's published value is its map
    // applied to its own carry in the same way, so the carry does not depend
    // on which predecessors had finished (results are reproducible).
    double carry[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) carry[c] = 0.0;
    if (tl > 0 && s_first != 0.0) {
        const int lim = t0[q];
        int base = T - 1, found = -1;
        for (;;) {
            int cnt = base - lim + 1;
            cnt = cnt < 64 ? cnt : 64;
            if (tid < cnt) s_win[tid] = wait_nonzero(&A.flag[base - tid], A.err, 17);
            __syncthreads();
            int m = -1;
            for (int L = 0; L < cnt; ++L)
                if (s_win[L] == 2) { m = L; break; }
            if (m >= 0) {
                found = base - m;
                break;
            }
            base -= cnt;
            __syncthreads();
            if (base < lim) {  // a phase's first tile always publishes its value
                atomicMax(A.err, 19);
                break;
            }
        }
        if (active && found >= 0) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) carry[c] = ld_dev(&A.tI[(int64_t)found * w + j0 + c]);
            for (int tk = found + 1; tk < T; ++tk) {
                const double pk = ld_dev(&A.tP[tk]);
#pragma unroll
                for (int c = 0; c < CPT; ++c)
                    carry[c] = fma(pk, carry[c], ld_dev(&A.tX[(int64_t)tk * w + j0 + c]));
            }
        }
    }

    // apply and store
    if (active) {
        double cv[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) cv[c] = carry[c];
#pragma unroll 1
        for (int q2 = 0; q2 < g; ++q2) {
            int o = q2 * A.lpr + jl;
            double pq = sP[o];
#pragma unroll
            for (int c = 0; c < CPT; ++c) cv[c] = pq * cv[c] + sX[o * CPT + c];
        }
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) cv[c] = av[i] * cv[c] + bv[i][c];
            const int r = row_of(i);
            if (r >= 0) store_cols_dev<CPT>(A.dst + (int64_t)r * w + j0, cv);
        }
        if (!incl_now && g == A.groups - 1) {  // value after the tile: its map applied to the carry
#pragma unroll
            for (int c = 0; c < CPT; ++c) st_dev(&A.tI[(int64_t)T * w + j0 + c], fma(Pt, carry[c], Xt[c]));
        }
    }
    stores_complete();
    __syncthreads();
    if (tid == 0) {
        if (!incl_now) st_dev(&A.flag[T], 2);
        st_dev(&A.flagw[T], 1);
    }
}

// --- narrow rows: rows as signals ------------------------------------------------
// For narrow rows (the HDP windows) the pass does without tile flags: the
// output rows start out holding a signalling-NaN pattern that no arithmetic
// produces, and a tile that gathers a row of the previous phase polls the row
// itself.  Rows that do not depend on the tile's carry-in (those at or after
// its first chain break) are stored as soon as they are known; the carry-in is
// the value of the last row of the preceding tile (read the same way), or,
// across a tile with no chain break, that tile's published map.  Maps are
// FP64, also marked unwritten until published.

// CPT labels of a row, once written (device-coherent loads, bounded poll).
template <int CPT>
__device__ __forceinline__ bool poll_cols(const float *p, float *v, int32_t *err, bool wait) {
    for (int it = 0;; ++it) {
        bool ok = true;
        if (CPT == 1) {
            uint32_t u = ld_dev(reinterpret_cast<const uint32_t *>(p));
            ok = u != kSentF;
            v[0] = __uint_as_float(u);
        } else {
#pragma unroll
            for (int h = 0; h < CPT / 2; ++h) {
                uint64_t u = ld_dev(reinterpret_cast<const uint64_t *>(p) + h);
                // unwritten: both halves hold the pattern (compared as 32-bit words)
                ok = ok && ((uint32_t)u != kSentF || (uint32_t)(u >> 32) != kSentF);
                v[2 * h] = __uint_as_float((uint32_t)u);
                v[2 * h + 1] = __uint_as_float((uint32_t)(u >> 32));
            }
        }
        if (ok || !wait) return ok;
        if (it > kSpinLimit) {
            atomicMax(err, 20);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Variants of the narrow-row pass: plain, fused matching, fused matching whose
// up pass reads the right image packed (8 bytes a pixel).
constexpr int kFuse = 1, kFusePacked = 2;

// FUSE: the up pass computes the cost of its rows (eq. E) instead of reading a
// cost volume, and the down pass reduces every row to its winning label.
// The down pass of the default narrow schedule (two labels per thread, four
// rows per group) is held to 80 VGPRs, as the up pass is by itself: six waves
// per SIMD, three tiles per compute unit.
template <bool UP, int CPT, int kRPG, int FUSE>
__global__ void __launch_bounds__(kNarrowThreads)
    __attribute__((amdgpu_waves_per_eu((!UP && CPT == 2 && kRPG == 4) ? 6 : 1)))
    k_pass_s(PassArgs A) {
    constexpr bool kWta = FUSE != 0 && !UP;
    constexpr int kSeg = kNarrowSegs;
    __shared__ double sP[kNarrowThreads];
    __shared__ double sX[kNarrowThreads * CPT];
    // segment maps: kSeg x (threads per row) products, then their columns
    // (sized by the launch for the row width)
    extern __shared__ double s_seg[];
    double *const sSegP = s_seg;
    double *const sSegX = s_seg + kSeg * A.lpr;
    __shared__ int s_ticket;
    __shared__ double s_first;
    __shared__ int32_t s_plan[P_WORDS];
    __shared__ float sWb[kWta ? kNarrowThreads * kRPG : 1];  // fused winner-takes-all candidates
    __shared__ int sWj[kWta ? kNarrowThreads * kRPG : 1];
    __shared__ int sWv[kWta ? kNarrowThreads * kRPG : 1];     // pixel of each row (lead threads)
    const int tid = threadIdx.x;
    // the ticket, and meanwhile the whole plan into LDS (one word per thread)
    if (tid == 0) s_ticket = atomicAdd(A.ticket, 1);
    if (tid < P_WORDS) s_plan[tid] = A.plan[tid];
    __syncthreads();
    const int T = s_ticket;
    const int K = s_plan[P_NPH];
    const int total = s_plan[UP ? P_TOT_UP : P_TOT_DN];
    if (T >= total) return;
    const int32_t *t0 = s_plan + (UP ? P_T0UP : P_T0DN);
    const int32_t *row0 = s_plan + P_ROW0;
    int q = 0;
    while (q + 1 < K && t0[q + 1] <= T) ++q;
    const int k = UP ? K - 1 - q : q;
    const int tl = T - t0[q];
    const int r0 = row0[k], r1 = row0[k + 1];
    const int w = A.width, rows = A.rows;
    const int g = tid / A.lpr, jl = tid - g * A.lpr;
    const int j0 = jl * CPT;
    const bool active = g < A.groups;

    // Stage 1: loads that do not depend on other tiles of this launch.  Every
    // load of the stage is issued before any loaded value is used: rows past
    // the end of the phase read a valid row of it instead and their results
    // are dropped, and the right-image reads of labels past the interval or
    // the image border read valid pixels whose values are not used.  So no
    // load waits behind a branch or behind another row's loads.
    int rr[kRPG], rc[kRPG];
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
        const int li = g * kRPG + i;
        const int r = UP ? r1 - 1 - (tl * rows + li) : r0 + tl * rows + li;
        const bool in = active && (UP ? r >= r0 : r < r1);
        rr[i] = in ? r : -1;
        rc[i] = in ? r : (UP ? r1 - 1 : r0);
    }
    // fused matching: pixel, column and interval of every row
    int fv[kRPG], fx[kRPG], flh[kRPG];
    if (FUSE) {
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
            fv[i] = at32(A.node, rc[i]);
            if (UP) fx[i] = at32(A.rx, rc[i]);
            flh[i] = at32(A.rlh, rc[i]);
        }
    }
    // Row maps x -> av * x + bv.  The constant terms are sums of non-negative
    // terms (costs, or coefficients times stored rows), so holding them in
    // FP32 adds one relative rounding of at most 2^-24 per row; the maps are
    // composed in FP64.  At most two light children per row are gathered (a
    // tree's root, its smallest pixel, has no upper or left tree neighbour).
    double av[kRPG];
    float bv[kRPG][CPT];
    int x0[kRPG], x1[kRPG];
    {
        float v[kRPG][CPT];
        uint8_t hf[kRPG];
        double sf[kRPG], of[kRPG];
        int pf[kRPG];
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
            const int r = rc[i];
            if (UP) {
                const int rn = r + 1 < r1 ? r + 1 : r;  // next row: heavy flag and coefficient
                hf[i] = at32(A.heavy, rn);
                sf[i] = at32(A.s, rn);
                x0[i] = at32(A.lc, r);
                x1[i] = at32(A.lc, A.n + r);
            } else {
                hf[i] = at32(A.heavy, r);
                sf[i] = at32(A.s, r);
                of[i] = at32(A.om, r);
                pf[i] = at32(A.prow, r);
            }
            if (!(FUSE && UP)) load_cols<CPT>(A.src + (int64_t)r * w + j0, v[i]);
        }
        if (FUSE && UP) {  // cost of labels lo + j0 .. (columns past hi hold 0), half of the rows at a time
            constexpr int kH = kRPG >= 2 ? 2 : 1;
            constexpr int kR2 = kRPG / kH;
#pragma unroll
            for (int h = 0; h < kH; ++h) {
                // right pixels packed (wide rows) or as FP32; each side
                // issues all its loads of the half before it uses any
                float4 Lp[kR2];
#pragma unroll
                for (int ii = 0; ii < kR2; ++ii) Lp[ii] = at32(A.imL, fv[h * kR2 + ii]);
                if (FUSE == kFusePacked) {
                    uint2 Rq[kR2][CPT];
#pragma unroll
                    for (int ii = 0; ii < kR2; ++ii) {
                        const int i = h * kR2 + ii;
                        const int a = flh[i] & 0xFFFF;
#pragma unroll
                        for (int c = 0; c < CPT; ++c)
                            Rq[ii][c] = at32(A.imRp, match_src(fv[i], fx[i], a + j0 + c));
                    }
#pragma unroll
                    for (int ii = 0; ii < kR2; ++ii) {
                        const int i = h * kR2 + ii;
                        const int a = flh[i] & 0xFFFF, b = flh[i] >> 16;
#pragma unroll
                        for (int c = 0; c < CPT; ++c) {
                            const int label = a + j0 + c;
                            const float4 Rp = packed_fallback(Rq[ii][c])
                                                  ? at32(A.imR, match_src(fv[i], fx[i], label))
                                                  : unpack_right(Rq[ii][c], A.rinv);
                            v[i][c] = label <= b ? match_cost_px(Lp[ii], Rp, fx[i] - label < 0, A.cp)
                                                 : 0.f;
                        }
                    }
                } else {
                    float4 Rp[kR2][CPT];
#pragma unroll
                    for (int ii = 0; ii < kR2; ++ii) {
                        const int i = h * kR2 + ii;
                        const int a = flh[i] & 0xFFFF;
#pragma unroll
                        for (int c = 0; c < CPT; ++c)
                            Rp[ii][c] = at32(A.imR, match_src(fv[i], fx[i], a + j0 + c));
                    }
#pragma unroll
                    for (int ii = 0; ii < kR2; ++ii) {
                        const int i = h * kR2 + ii;
                        const int a = flh[i] & 0xFFFF, b = flh[i] >> 16;
#pragma unroll
                        for (int c = 0; c < CPT; ++c) {
                            const int label = a + j0 + c;
                            v[i][c] = label <= b ? match_cost_px(Lp[ii], Rp[ii][c], fx[i] - label < 0, A.cp)
                                                 : 0.f;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
            const bool in = rr[i] >= 0;
            const int r = rc[i];
            if (UP) {
                av[i] = !in ? 1.0 : (r + 1 < r1 && hf[i]) ? sf[i] : 0.0;
#pragma unroll
                for (int c = 0; c < CPT; ++c) bv[i][c] = in ? v[i][c] : 0.f;
                if (!in) x0[i] = x1[i] = -1;
            } else {
                av[i] = !in ? 1.0 : hf[i] ? sf[i] : 0.0;
#pragma unroll
                for (int c = 0; c < CPT; ++c) bv[i][c] = in ? (float)(of[i] * (double)v[i][c]) : 0.f;
                x0[i] = (in && !hf[i]) ? pf[i] : -1;
                x1[i] = -1;
            }
        }
    }
    // The up pass marks as unwritten its rows of the down pass's output that
    // the down pass's tiles poll: parents of a chain head (a light child) and
    // the last row of every down tile.  The marks are stored when the tile is
    // done with everything else (the down pass is a later launch).
    uint32_t fill_mask = 0;
    if (UP && A.fill) {
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
            const int r = rr[i];
            if (r >= 0 && (x0[i] >= 0 || (r - r0 + 1) % rows == 0)) fill_mask |= 1u << i;
        }
    }
    auto mark_fill = [&]() {
        if (!UP || !fill_mask) return;
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
            if (!(fill_mask >> i & 1u)) continue;
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                reinterpret_cast<uint32_t *>(A.fill)[(int64_t)rr[i] * w + j0 + c] = kSentF;
        }
    };

    // Stage 2: gather the rows of the previous phase, half of the rows at a
    // time (fewer registers in flight).  The first read of every gathered row
    // (and its coefficient) of the half is issued at once, for the rows that
    // exist only (device-coherent reads are not spent on absent children); a
    // row that is still unwritten is then polled on its own.
    {
        constexpr int kG = UP ? 2 : 1;  // gathered rows per row
        constexpr int kH = kRPG >= 2 ? 2 : 1;
        constexpr int kR2 = kRPG / kH;
#pragma unroll
        for (int h = 0; h < kH; ++h) {
            float gv[kR2][kG][CPT];
            double gs[kR2][kG];
            bool ok[kR2][kG];
#pragma unroll
            for (int ii = 0; ii < kR2; ++ii) {
                const int i = h * kR2 + ii;
#pragma unroll
                for (int m = 0; m < kG; ++m) {
                    const int x = m == 0 ? x0[i] : x1[i];
                    ok[ii][m] = true;
                    gs[ii][m] = 0.0;
#pragma unroll
                    for (int c = 0; c < CPT; ++c) gv[ii][m][c] = 0.f;
                    if (x >= 0) {
                        gs[ii][m] = UP ? at32(A.s, x) : at32(A.s, rc[i]);
                        ok[ii][m] = poll_cols<CPT>(A.dst + (int64_t)x * w + j0, gv[ii][m], A.err, false);
                    }
                }
            }
#pragma unroll
            for (int ii = 0; ii < kR2; ++ii) {
                const int i = h * kR2 + ii;
#pragma unroll
                for (int m = 0; m < kG; ++m) {
                    const int x = m == 0 ? x0[i] : x1[i];
                    if (x < 0) continue;
                    if (!ok[ii][m]) poll_cols<CPT>(A.dst + (int64_t)x * w + j0, gv[ii][m], A.err, true);
#pragma unroll
                    for (int c = 0; c < CPT; ++c)
                        bv[i][c] = (float)((double)bv[i][c] + gs[ii][m] * (double)gv[ii][m][c]);
                }
            }
        }
    }

    // maps of this thread's rows, of the groups before it and of the tile
    double P = 1.0, X[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) X[c] = 0.0;
#pragma unroll
    for (int i = 0; i < kRPG; ++i) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) X[c] = av[i] * X[c] + bv[i][c];
        P *= av[i];
    }
    if (tid == 0) s_first = av[0];
    sP[tid] = P;
#pragma unroll
    for (int c = 0; c < CPT; ++c) sX[tid * CPT + c] = X[c];
    __syncthreads();
    // Exclusive map of the groups before this thread's group (Pg, Xg) and the
    // tile map (Pt, Xt), in two levels: the groups are cut into kSeg segments
    // scanned at the same time, then the segment maps are combined.
    const int seg_len = (A.groups + kSeg - 1) / kSeg;
    const int sg = g / seg_len;
    double Pg = 1.0, Xg[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) Xg[c] = 0.0;
    if (active) {
        const int q_end = min((sg + 1) * seg_len, A.groups);
        double Ps = 1.0, Xs[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) Xs[c] = 0.0;
        for (int q2 = sg * seg_len; q2 < q_end; ++q2) {
            if (q2 == g) {
                Pg = Ps;
#pragma unroll
                for (int c = 0; c < CPT; ++c) Xg[c] = Xs[c];
            }
            int o = q2 * A.lpr + jl;
            double pq = sP[o];
#pragma unroll
            for (int c = 0; c < CPT; ++c) Xs[c] = pq * Xs[c] + sX[o * CPT + c];
            Ps *= pq;
        }
        if (g == q_end - 1) {  // the segment's last group publishes the segment map
            sSegP[sg * A.lpr + jl] = Ps;
#pragma unroll
            for (int c = 0; c < CPT; ++c) sSegX[(sg * A.lpr + jl) * CPT + c] = Xs[c];
        }
    }
    __syncthreads();
    double Pt = 1.0, Xt[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) Xt[c] = 0.0;
    if (active) {
        const int nseg = (A.groups + seg_len - 1) / seg_len;
#pragma unroll 1
        for (int q2 = 0; q2 < nseg; ++q2) {
            if (q2 == sg) {  // segments before this one, then this group's offset in it
#pragma unroll
                for (int c = 0; c < CPT; ++c) Xg[c] = Pg * Xt[c] + Xg[c];
                Pg *= Pt;
            }
            int o = q2 * A.lpr + jl;
            double pq = sSegP[o];
#pragma unroll
            for (int c = 0; c < CPT; ++c) Xt[c] = pq * Xt[c] + sSegX[o * CPT + c];
            Pt *= pq;
        }
    }
    // a tile without a chain break publishes its map for the tiles after it
    if (active && g == 0 && Pt != 0.0 && tl > 0) {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            st_dev(reinterpret_cast<uint64_t *>(&A.tXs[(int64_t)T * w + j0 + c]),
                   (uint64_t)__double_as_longlong(Xt[c]));
        // The product word doubles as the map's flag, so it is stored after
        // every word of the map has completed (group 0 is in one wavefront,
        // whose outstanding stores all complete at this wait).
        stores_complete();
        if (jl == 0)
            st_dev(reinterpret_cast<uint64_t *>(&A.tPs[T]), (uint64_t)__double_as_longlong(Pt));
    }
    // fused winner-takes-all: per row, this thread's least value and its column
    // (first of equal values), taken into LDS as the row is stored (every row
    // of the tile is stored exactly once).  Each row's interval is kept
    // packed, lo | hi << 8, two rows per register.
    uint32_t lh2[(kRPG + 1) / 2];
    if (kWta) {
        if (jl == 0) {
#pragma unroll
            for (int i = 0; i < kRPG; ++i) sWv[tid * kRPG + i] = fv[i];
        }
#pragma unroll
        for (int i = 0; i < (kRPG + 1) / 2; ++i) lh2[i] = 0;
#pragma unroll
        for (int i = 0; i < kRPG; ++i)
            lh2[i >> 1] |= ((uint32_t)(flh[i] & 0xFF) | (uint32_t)((flh[i] >> 16) & 0xFF) << 8)
                           << (16 * (i & 1));
    }
    auto take = [&](int i, const double *cv) {
        const uint32_t lh = (lh2[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
        const int nl = (int)(lh >> 8) - (int)(lh & 0xFF);  // last valid column
        float best = __builtin_inff();
        int bj = 0x7fffffff;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const float x = (float)cv[c];
            if (j0 + c <= nl && x < best) {
                best = x;
                bj = j0 + c;
            }
        }
        sWb[tid * kRPG + i] = best;
        sWj[tid * kRPG + i] = bj;
    };
    // rows at or after the tile's first chain break do not depend on the carry-in
    if (active) {
        double cv[CPT], pp = Pg;
#pragma unroll
        for (int c = 0; c < CPT; ++c) cv[c] = Xg[c];
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) cv[c] = av[i] * cv[c] + bv[i][c];
            pp *= av[i];
            if (pp == 0.0 && rr[i] >= 0) {
                store_cols_dev<CPT>(A.dst + (int64_t)rr[i] * w + j0, cv);
                if (kWta) take(i, cv);
            }
        }
    }
    const bool carried = !(tl == 0 || s_first == 0.0 || !active);
    if (!kWta && !carried) {  // every row was carry-independent
        mark_fill();
        return;
    }

    if (carried) {
        // Carry-in: the last row of the preceding tile, or across tiles without
        // a chain break (whose maps are published) the last row of an earlier
        // tile with those maps applied forward one tile at a time, rounded as
        // a stored row.  Such a tile stores its last row the same way (its map
        // applied to its carry), so the carry does not depend on which path
        // was taken (results are reproducible).
        double carry[CPT];
        {
            const int lim = t0[q];
            int pred = T - 1;
            for (int it = 0;; ++it) {
                // row processed just before tile pred + 1 of this phase
                const int nxt = pred + 1 - lim;
                const int lr = UP ? r1 - nxt * rows : r0 + nxt * rows - 1;
                float v[CPT];
                if (poll_cols<CPT>(A.dst + (int64_t)lr * w + j0, v, A.err, false)) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) carry[c] = (double)v[c];
                    for (int tk = pred + 1; tk < T; ++tk) {
                        // (a batch's tile maps take far less than 4 GiB)
                        const double pk = __longlong_as_double((long long)ld_dev32(
                            reinterpret_cast<const uint64_t *>(A.tPs), (uint32_t)tk));
#pragma unroll
                        for (int c = 0; c < CPT; ++c) {
                            const double xk = __longlong_as_double((long long)ld_dev32(
                                reinterpret_cast<const uint64_t *>(A.tXs), (uint32_t)(tk * w + j0 + c)));
                            carry[c] = (double)(float)fma(pk, carry[c], xk);
                        }
                    }
                    break;
                }
                if (pred > lim) {  // map of tile pred published: look one tile further back
                    // (its product word is stored once the whole map is written)
                    const bool ok =
                        ld_dev(reinterpret_cast<const uint64_t *>(&A.tPs[pred])) != kSentD;
                    if (ok) {
                        --pred;
                        continue;
                    }
                }
                if (it > kSpinLimit) {
                    atomicMax(A.err, 21);
#pragma unroll
                    for (int c = 0; c < CPT; ++c) carry[c] = 0.0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }

        // rows before the first chain break, with the carry-in; in a tile
        // without a break the last row is the tile map applied to the carry
        double cv[CPT], pp = Pg;
#pragma unroll
        for (int c = 0; c < CPT; ++c) cv[c] = Pg * carry[c] + Xg[c];
#pragma unroll
        for (int i = 0; i < kRPG; ++i) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) cv[c] = av[i] * cv[c] + bv[i][c];
            pp *= av[i];
            if (pp != 0.0 && rr[i] >= 0) {
                if (Pt != 0.0 && g == A.groups - 1 && i == kRPG - 1) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) cv[c] = fma(Pt, carry[c], Xt[c]);
                }
                store_cols_dev<CPT>(A.dst + (int64_t)rr[i] * w + j0, cv);
                if (kWta) take(i, cv);
            }
        }
    }

    if (kWta) {
        // The row's threads are consecutive and later threads hold later
        // columns: a tree over them in LDS (at step s, thread jl with jl a
        // multiple of 2s takes the candidate of thread jl + s only if it is
        // strictly smaller) leaves each row's first least value with its lead
        // thread.  Every row of the tile is combined at each step.
        __syncthreads();
        for (int s2 = 1; s2 < A.lpr; s2 <<= 1) {
            if (active && (jl & (2 * s2 - 1)) == 0 && jl + s2 < A.lpr) {
#pragma unroll
                for (int i = 0; i < kRPG; ++i) {
                    const float x = sWb[(tid + s2) * kRPG + i];
                    if (x < sWb[tid * kRPG + i]) {
                        sWb[tid * kRPG + i] = x;
                        sWj[tid * kRPG + i] = sWj[(tid + s2) * kRPG + i];
                    }
                }
            }
            __syncthreads();
        }
        if (active && jl == 0) {
#pragma unroll
            for (int i = 0; i < kRPG; ++i)
                if (rr[i] >= 0)
                    A.disp[sWv[tid * kRPG + i]] =
                        (int)((lh2[i >> 1] >> (16 * (i & 1))) & 0xFF) + sWj[tid * kRPG + i];
        }
    }
    mark_fill();
}

// --- workspace --------------------------------------------------------------------

struct AggWs {
    int32_t *plan, *ticket, *flags;  // flags: kPassSets x (flag[tiles], flagw[tiles])
    double *s, *om, *tP, *tX, *tI;
    double *tPs, *tXs;  // narrow rows: kPassSets x tile maps (tiles, tiles x width)
    uint2 *imRp;    // right image packed for the fused up pass
    float *up;      // U when the caller does not keep it
    float *ug;      // U of the gradient (backward)
    double *red;    // per-block partial sums (backward)
    int64_t tiles;
};

// Upper bound on the tiles of any valid schedule (fewest rows per tile).
static int64_t max_tiles(int64_t n, int width) {
    return n / make_geom(width, 1, 4).rows + HDP_MAX_PHASES + 2;
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
    a.tiles = nt;
    a.plan = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * P_WORDS));
    a.ticket = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * kPassSets));
    a.flags = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 2 * kPassSets * nt));
    a.s = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.om = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.tP = reinterpret_cast<double *>(take(sizeof(double) * nt));
    a.tX = reinterpret_cast<double *>(take(sizeof(double) * nt * width));
    a.tI = reinterpret_cast<double *>(take(sizeof(double) * nt * width));
    const bool narrow = narrow_rows(width);  // one block: the prologue marks it in one sweep
    a.tPs = reinterpret_cast<double *>(
        take(narrow ? sizeof(double) * kPassSets * nt * (width + 1) : 8));
    a.tXs = a.tPs + (narrow ? kPassSets * nt : 0);
    a.imRp = reinterpret_cast<uint2 *>(take(sizeof(uint2) * n));
    a.up = reinterpret_cast<float *>(take(sizeof(float) * n * width));
    a.ug = reinterpret_cast<float *>(take(sizeof(float) * n * width));
    // partial sums of the adjoint: one per block of the edge gradients (at most
    // n / 4 + 1 with 4 lanes per row and 256 threads), then one per summing block
    a.red = reinterpret_cast<double *>(take(sizeof(double) * (n / 4 + 64 + kSumBlocks)));
    *bytes = off + 256;
    return a;
}

size_t aggregate_workspace_bytes(int64_t n, int width) {
    size_t b = 0;
    carve_agg_ws(nullptr, n, width, &b);
    return b;
}

// FUSE (narrow rows only): the fused matching variant of the narrow-row pass
// (kFusePacked: its up pass reads the packed right image).
template <bool UP, int CPT, int RPG, int FUSE>
static void launch_pass(const PassArgs &A, int64_t tiles, hipStream_t st) {
    timer_before(UP ? HDP_TIMER_UP_PASS : HDP_TIMER_DOWN_PASS, st);
    if (FUSE || narrow_rows(A.width)) {
        const size_t seg = sizeof(double) * kNarrowSegs * A.lpr * (1 + CPT);
        k_pass_s<UP, CPT, RPG, FUSE><<<(unsigned)tiles, kNarrowThreads, seg, st>>>(A);
    } else {
        k_pass<UP, CPT, RPG><<<(unsigned)tiles, kBlock, 0, st>>>(A);
    }
    timer_after(UP ? HDP_TIMER_UP_PASS : HDP_TIMER_DOWN_PASS, st);
}

// One pass with flag set `set` (cleared by the prologue of this call).
template <bool UP, int FUSE = 0>
static void run_pass(PassArgs A, const AggWs &w, const TileGeom &tg, int set, hipStream_t st,
                     float *fill = nullptr) {
    int64_t tiles = A.n / tg.rows + HDP_MAX_PHASES + 2;  // >= the plan's tile count
    A.ticket = w.ticket + set;
    A.flag = w.flags + (int64_t)(2 * set) * w.tiles;
    A.flagw = w.flags + (int64_t)(2 * set + 1) * w.tiles;
    A.tPs = w.tPs + (int64_t)set * w.tiles;
    A.tXs = w.tXs + (int64_t)set * w.tiles * A.width;
    A.fill = fill;
    if (tg.cpt == 4) {
        if (tg.rpg == 4) launch_pass<UP, 4, 4, FUSE>(A, tiles, st);
        else launch_pass<UP, 4, 8, FUSE>(A, tiles, st);
    } else if (tg.cpt == 2) {
        if (tg.rpg == 4) launch_pass<UP, 2, 4, FUSE>(A, tiles, st);
        else if (tg.rpg == 8) launch_pass<UP, 2, 8, FUSE>(A, tiles, st);
        else launch_pass<UP, 2, 16, FUSE>(A, tiles, st);
    } else {
        if (tg.rpg == 4) launch_pass<UP, 1, 4, FUSE>(A, tiles, st);
        else launch_pass<UP, 1, 8, FUSE>(A, tiles, st);
    }
}

static PassArgs pass_args(const hdp_forest &f, int width, const AggWs &w, const TileGeom &tg) {
    PassArgs A{};
    A.n = (int)f.n;
    A.width = width;
    A.lpr = tg.lpr;
    A.groups = tg.groups;
    A.rows = tg.rows;
    A.s = w.s;
    A.om = w.om;
    A.heavy = f.heavy;
    A.prow = f.prow;
    A.lc = f.lc;
    A.plan = w.plan;
    A.tP = w.tP;
    A.tX = w.tX;
    A.tI = w.tI;
    A.err = f.info + HDP_INFO_ERROR;
    return A;
}

// Coefficients and the plan of both passes (device side, no host sync).
// fill0 / fill1: outputs of the up passes of this call (narrow rows only).
static void prologue(const hdp_forest &f, int width, float sigma, const AggWs &w, hipStream_t st,
                     float *fill0 = nullptr, float *fill1 = nullptr,
                     const float *right = nullptr, float rscale = 1.f) {
    const bool narrow = narrow_rows(width);
    int64_t m = f.n > w.tiles ? f.n : w.tiles;
    // narrow rows: the product words of the tile maps, marked unpublished
    int64_t map_words = narrow ? (int64_t)kPassSets * w.tiles : 0;
    k_prologue<<<grid_for(m), kBlock, 0, st>>>(
        f.n, f.rw, f.prow, f.heavy, 1.0 / (double)sigma, w.s, w.om, w.flags, w.tiles, w.ticket,
        f.phase_ptr, f.info, tile_geom(width).rows, w.plan,
        narrow ? reinterpret_cast<uint32_t *>(fill0) : nullptr,
        narrow ? reinterpret_cast<uint32_t *>(fill1) : nullptr, width,
        reinterpret_cast<uint64_t *>(w.tPs), map_words, reinterpret_cast<const float4 *>(right),
        right ? w.imRp : nullptr, rscale);
}

// Two passes of `src` over the forest: U -> up, A -> out (flag sets up_set, up_set + 1).
static void two_pass(const hdp_forest &f, int width, const float *src, float *up, float *out,
                     const AggWs &w, int up_set, hipStream_t st) {
    TileGeom tg = tile_geom(width);
    PassArgs A = pass_args(f, width, w, tg);
    A.src = src;
    A.dst = up;
    run_pass<true>(A, w, tg, up_set, st, out);
    A.src = up;
    A.dst = out;
    run_pass<false>(A, w, tg, up_set + 1, st);
}

void launch_aggregate(const hdp_forest &f, int width, const float *cost, float sigma, float *agg,
                      float *up, void *ws, hipStream_t st) {
    size_t bytes;
    AggWs w = carve_agg_ws(ws, f.n, width, &bytes);
    float *U = up ? up : w.up;
    prologue(f, width, sigma, w, st, U);
    two_pass(f, width, cost, U, agg, w, 0, st);
}

// Rows of at least this many labels take the right image packed in the fused up pass.
constexpr int kPackRightMinWidth = 64;

// Cost, aggregation and winner-takes-all of one layer.  Narrow rows: the two
// fused passes (no cost volume in memory, no separate WTA launch).  Wide rows:
// the cost volume is built in the workspace and the three steps run apart.
void launch_match(const float *left, const float *right, const LevelGeom &g, const hdp_forest &f,
                  int width, const hdp_cost_params &p, float sigma, float *agg, int32_t *disp,
                  void *ws, hipStream_t st) {
    size_t bytes;
    AggWs w = carve_agg_ws(ws, f.n, width, &bytes);
    if (!narrow_rows(width)) {
        launch_cost_volume(left, right, g, f.node, f.lo, f.hi, width, p, w.ug, st);
        prologue(f, width, sigma, w, st, w.up);
        two_pass(f, width, w.ug, w.up, agg, w, 0, st);
        launch_wta(g, f.node, f.lo, f.hi, width, agg, disp, st);
        return;
    }
    // Rows of many labels read the right image packed (8 bytes a pixel), so
    // that the right-pixel reads, most of the up pass's traffic there, take
    // half the bytes; the narrow HDP windows (where the pass is bound by its
    // dependency chain, not by these reads) read it as it is (measured).
    const bool pack = width >= kPackRightMinWidth;
    const float rscale = ldexpf(1.0f, 2 * g.level);
    prologue(f, width, sigma, w, st, w.up, nullptr, pack ? right : nullptr, rscale);
    TileGeom tg = tile_geom(width);
    PassArgs A = pass_args(f, width, w, tg);
    A.imL = reinterpret_cast<const float4 *>(left);
    A.imR = reinterpret_cast<const float4 *>(right);
    A.imRp = pack ? w.imRp : nullptr;
    A.rinv = 1.0f / rscale;
    A.cp = CostParams{p.a_c, p.tau_c, p.a_g, p.tau_g, p.border};
    A.node = f.node;
    A.rx = f.rx;
    A.rlh = f.rlh;
    A.disp = disp;
    A.src = nullptr;
    A.dst = w.up;
    if (pack)
        run_pass<true, kFusePacked>(A, w, tg, 0, st, agg);
    else
        run_pass<true, kFuse>(A, w, tg, 0, st, agg);
    A.src = w.up;
    A.dst = agg;
    run_pass<false, kFuse>(A, w, tg, 1, st);
}

// --- adjoint ----------------------------------------------------------------------------

// Per row (edge to the parent): acc = sum_x [Ug (Ac(p) - s Uc) + Uc (Ag(p) - s Ug)];
// grad_w = -(s/sigma) acc; per-block partial of acc * s * w / sigma^2.  LPR
// consecutive lanes take one row (lane j reads labels j, j + LPR, ...: the
// row's labels are read by consecutive lanes), so a wavefront covers 64 / LPR
// rows; the row sum is a butterfly over its LPR lanes.
template <int LPR>
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
    const int64_t r = gtid() / LPR;
    const int j = (int)(threadIdx.x & (LPR - 1));
    double contrib = 0.0;
    int p = -1;
    double sr = 0.0;
    double acc = 0.0;
    if (r < n) {
        p = prow[r];
        sr = s[r];
        if (p >= 0) {
            const float *ucr = uc + r * width, *ugr = ug + r * width;
            const float *acp = ac + (int64_t)p * width, *agp = ag + (int64_t)p * width;
            for (int x = j; x < width; x += LPR) {
                const double u1 = ucr[x], u2 = ugr[x];
                acc += u2 * ((double)acp[x] - sr * u1) + u1 * ((double)agp[x] - sr * u2);
            }
        }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (r < n && j == 0) {
        if (grad_w) grad_w[node[r]] = p >= 0 ? (float)(-(sr * inv_sigma) * acc) : 0.f;
        if (p >= 0) contrib = acc * sr * (double)rw[r] * inv_sigma * inv_sigma;
    }
    // block partial in a fixed order: rows of a wavefront, then wavefronts
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += part[k];
        red[blockIdx.x] = t;
    }
}

// Sum of nb partials: every block sums a strided share (fixed order), the
// last launch has one block and writes the float result.
__global__ void __launch_bounds__(kBlock) k_sum_red(const double *__restrict__ red, int64_t nb,
                                                    double *__restrict__ out2,
                                                    float *__restrict__ out) {
    __shared__ double sh[kBlock];
    double t = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = gtid(); i < nb; i += stride) t += red[i];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (out) *out = (float)sh[0];
        else out2[blockIdx.x] = sh[0];
    }
}

// Launch of the edge gradients with the row width's lanes per row.
static int64_t launch_edge_grad(const hdp_forest &f, int width, const double *s, const float *uc,
                                const float *ac, const float *ug, const float *ag,
                                double inv_sigma, float *grad_w, double *red, hipStream_t st) {
    const int lpr = width <= 8 ? 4 : width <= 16 ? 8 : width <= 32 ? 16 : width <= 64 ? 32 : 64;
    const int64_t nb = (f.n * lpr + kBlock - 1) / kBlock;
#define HDP_EDGE_GRAD(L)                                                                           \
    k_edge_grad<L><<<(unsigned)nb, kBlock, 0, st>>>(f.n, width, f.prow, f.node, f.rw, s, uc, ac,  \
                                                    ug, ag, inv_sigma, grad_w, red)
    if (lpr == 4) HDP_EDGE_GRAD(4);
    else if (lpr == 8) HDP_EDGE_GRAD(8);
    else if (lpr == 16) HDP_EDGE_GRAD(16);
    else if (lpr == 32) HDP_EDGE_GRAD(32);
    else HDP_EDGE_GRAD(64);
#undef HDP_EDGE_GRAD
    return nb;
}

// Partial sums of the edge gradients -> dL/dsigma (two launches, fixed order).
static void launch_sum(const double *red, int64_t nb, double *red2, float *out, hipStream_t st) {
    const int64_t blocks = (nb + kBlock - 1) / kBlock < kSumBlocks ? (nb + kBlock - 1) / kBlock
                                                                   : kSumBlocks;
    k_sum_red<<<(unsigned)blocks, kBlock, 0, st>>>(red, nb, red2, nullptr);
    k_sum_red<<<1, kBlock, 0, st>>>(red2, blocks, nullptr, out);
}

void launch_aggregate_backward(const hdp_forest &f, int width, const float *cost, const float *agg,
                               const float *up, const float *grad_agg, float sigma,
                               float *grad_cost, float *grad_w, float *grad_sigma, void *ws,
                               hipStream_t st) {
    size_t bytes;
    AggWs w = carve_agg_ws(ws, f.n, width, &bytes);
    prologue(f, width, sigma, w, st, w.ug, up ? nullptr : w.up);
    const float *uc = up;
    if (!uc) {  // recompute the up pass of the cost
        TileGeom tg = tile_geom(width);
        PassArgs A = pass_args(f, width, w, tg);
        A.src = cost;
        A.dst = w.up;
        run_pass<true>(A, w, tg, 2, st);
        uc = w.up;
    }
    two_pass(f, width, grad_agg, w.ug, grad_cost, w, 0, st);
    if (grad_w || grad_sigma) {
        const int64_t nb = launch_edge_grad(f, width, w.s, uc, agg, w.ug, grad_cost,
                                            1.0 / (double)sigma, grad_w, w.red, st);
        if (grad_sigma) launch_sum(w.red, nb, w.red + nb, grad_sigma, st);
    }
}

}  // namespace hdp
