// Spanning forest of a pyramid layer (Section 1; Section 3.2 Rules 1-2 and
// DT-Rules 1-2 in the exact regime), rooting, level order and the chain-phase
// schedule of the aggregation.
//
// Pipeline (all on the device, fixed launch counts, early exit on convergence):
//   1. edge keys  k = 4^level * max_c |dI_c|, edge id 2p (right) / 2p+1 (down);
//      an edge whose two pixel intervals differ is dropped (in the regime
//      DT-Rule 2 admits only equal intervals; DT-Rule 1 is then implied);
//   2. Boruvka rounds: every component takes its least (k, id) edge with a
//      64-bit atomicMin, components hook along it (a mutual pair keeps the
//      smaller id as root), hook pointers are followed to the root.  With
//      unique (k, id) keys the result is the unique minimum spanning forest,
//      i.e. the same forest as Kruskal's process;
//   3. each tree is rooted at its smallest pixel id;
//   4. Euler tour (neighbour order right, down, left, up) ranked by in-place
//      pointer jumping on packed (next, distance) words -> parent, subtree size;
//   5. heavy child = child of largest subtree (smallest id on ties);
//   6. one prefix sum over the concatenated tours -> depth, light depth and
//      preorder of every pixel;
//   7. rows of the volume layout: pixels in preorder, stably partitioned by
//      light depth (each heavy path becomes a contiguous run of rows);
//   8. canonical level order (depth, id) by a stable radix sort.
#include "common.hpp"
#include "kernels.hpp"
#include "sortscan.hpp"

namespace hdp {

constexpr uint32_t kNoKey = 0xFFFFFFFFu;
constexpr uint64_t kNoEdge = ~0ull;

enum {
    FLAG_BV = 0,      // [64] hooking happened in Boruvka round r
    FLAG_RANK = 64,   // [64] pointer jumping not yet converged after round r
    FLAG_WORDS = 128
};

enum {
    CTR_E = 0,      // live edges after the tile-local phase
    CTR_RALL = 1,   // active components after the tile-local phase
    CTR_ET = 2,     // edges left for the one-workgroup tail
    CTR_RUNS = 3,   // run ends of the tile-local tour ranking
    CTR_AT = 4,     // run ends left for the one-workgroup tail
    kCounters = 8
};

// Rounds run by full-grid launches before one workgroup finishes the rest.
constexpr int kBvGridRounds = 4;
// Further rounds on the compacted list of live edges (cheap: a pass over the
// few edges still live), before the one-workgroup tail takes what is left.
constexpr int kBvListRounds = 8;
// Pointer-jumping steps on the full grid are taken kRankJumps per launch.  A
// layer without intervals (one spanning tree per pair) gets as many launches
// as its longest possible list needs: entries stay open until their pointer
// reaches the list end, so stopping early would leave the one-workgroup tail
// nearly the whole list of a large tree.
constexpr int kRankJumps = 12;
// Sizes of the one-workgroup LDS tails: spanning forest (edges, components,
// hash slots; endpoints and component state are 16-bit indices) and tour
// ranking (list entries).
constexpr int kTE = 6144, kTN = 3072, kTH = 4096;
constexpr int64_t kTopAloneBorderPx = 2 * kTE / 3;
constexpr int kTailEdgesPerThread = kTE / 1024;
constexpr int kTA = 8192;
// A contracted graph of at most kTE live edges, or a contracted tour list of
// at most kTA entries, skips the full-grid rounds and goes straight to its tail.

// --- shared helpers ------------------------------------------------------------------

constexpr int kLocalThreads = 1024;  // one workgroup per tile, one thread per pixel
constexpr int kTilePx = kTile * kTile;
constexpr int kHalo = kTile + 2;      // a tile with a one-pixel border
constexpr int kGridCap = 2048;       // workgroups of the grid-stride list kernels

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier for a workgroup that exchanges data through device-coherent global
// memory: every wave's memory operations complete before the barrier.
__device__ __forceinline__ void wg_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// One step of a wavefront minimum: each lane takes the smaller of its value
// and the value the DPP pattern kCtrl moves to it (rows outside kRowMask, and
// disabled source lanes, contribute the identity ~0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_min_step(uint64_t v) {
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t slo = (uint32_t)__builtin_amdgcn_update_dpp(-1, lo, kCtrl, kRowMask, 0xF, false);
    const uint32_t shi = (uint32_t)__builtin_amdgcn_update_dpp(-1, hi, kCtrl, kRowMask, 0xF, false);
    const uint64_t o = ((uint64_t)shi << 32) | slo;
    return o < v ? o : v;
}

// Minimum of v over the 64 lanes of the wavefront (all lanes active), by DPP
// row steps without LDS: within quads, half rows and rows, then across rows
// with the row broadcasts; lane 63 ends with the total.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    v = dpp_min_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_min_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_min_step<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_min_step<0x140, 0xF>(v);  // row_mirror
    v = dpp_min_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_min_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Slot in a list for each lane with pred set: one atomic per wavefront.
__device__ __forceinline__ int wave_append(bool pred, int32_t *count) {
    uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader, 64);
    return base + __popcll(m & lanemask_lt());
}

struct TileInfo {
    int pair, x0, y0, tw, th, W, H, base;
};

__device__ __forceinline__ TileInfo tile_info(const LevelGeom &g, int t) {
    int lo = 0, hi = g.n_pairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (g.toff[mid] <= t) lo = mid; else hi = mid - 1;
    }
    TileInfo ti;
    ti.pair = lo;
    ti.W = g.W[lo];
    ti.H = g.H[lo];
    ti.base = g.off[lo];
    int k = t - g.toff[lo];
    int ntx = (ti.W + kTile - 1) / kTile;
    int ty = k / ntx;
    ti.x0 = (k - ty * ntx) * kTile;
    ti.y0 = ty * kTile;
    ti.tw = min(kTile, ti.W - ti.x0);
    ti.th = min(kTile, ti.H - ti.y0);
    return ti;
}

__device__ __forceinline__ int64_t tile_pixel(const TileInfo &t, int i) {
    return t.base + (int64_t)(t.y0 + (i >> 5)) * t.W + t.x0 + (i & (kTile - 1));
}

// Per-pixel kernels whose scattered stores land in per-tile ranges (tour
// positions, preorder) walk the image tile by tile: four kBlock-thread blocks
// per 32x32 tile, and the blocks of one tile on one XCD (blocks are dealt to
// the 8 XCDs in turn), so each range is written through one L2.
static_assert(kTilePx == 4 * kBlock, "four blocks per tile");
__device__ __forceinline__ int64_t tiled_pixel(const LevelGeom &g, int n_tiles, int *W,
                                               bool *ok) {
    const int b = blockIdx.x, xcd = b % kXcds, k = b / kXcds;
    const int tile = (k >> 2) * kXcds + xcd;
    *ok = false;
    *W = 1;
    if (tile >= n_tiles) return 0;
    const TileInfo t = tile_info(g, tile);
    const int ly = (k & 3) * (kBlock / kTile) + (int)threadIdx.x / kTile;
    const int lx = (int)threadIdx.x & (kTile - 1);
    *ok = lx < t.tw && ly < t.th;
    *W = t.W;
    return tile_pixel(t, ly * kTile + lx);
}
inline unsigned tiled_grid(int n_tiles) { return 4u * kXcds * (unsigned)((n_tiles + kXcds - 1) / kXcds); }

// Integer edge key 4^level * max_c |dI_c| (exact: level images hold dyadic means).
__device__ __forceinline__ uint32_t edge_key(float4 a, float4 b, float scale) {
    float m = fmaxf(fmaxf(fabsf(a.x - b.x), fabsf(a.y - b.y)), fabsf(a.z - b.z));
    return __float2uint_rn(m * scale);
}

__device__ __forceinline__ bool same_interval(const int32_t *plo, const int32_t *phi, int64_t v,
                                              int64_t q) {
    return !plo || (plo[v] == plo[q] && phi[v] == phi[q]);
}

__device__ __forceinline__ uint64_t key64(uint32_t k, int64_t eid) {
    return ((uint64_t)k << 32) | (uint64_t)(uint32_t)eid;
}

__global__ void k_tree_init(int32_t *__restrict__ flags, int32_t *__restrict__ ctr,
                            int32_t *__restrict__ info) {
    int t = threadIdx.x;
    if (t < FLAG_WORDS) flags[t] = 0;
    if (t < kCounters) ctr[t] = 0;
    if (t < HDP_INFO_WORDS) info[t] = 0;
}

// --- 1-2. spanning forest: tile-local phase ---------------------------------------
// Every kTile x kTile tile runs Boruvka in LDS on its own pixels.  A local
// component hooks only along its least (key, id) incident edge over ALL its
// edges, including those that leave the tile; when that edge leaves the tile
// the component waits for the global phase.  By the cut property every edge
// taken is an edge of the minimum spanning forest, and when the loop stops
// every component that still has an incident edge owns a pixel on the tile
// border, which bounds the work left to the global rounds.
//
// Components are named by the pixel id of their local root.  cw[x] packs the
// parent link of component x: low 32 bits the parent (x itself for a root),
// high 32 bits 0 for a permanent link or r + 1 for a hook made in round r.

// Slots of the per-tile table of component pairs (at most 2 * kTilePx live
// edges inside a tile, so the table never needs more).
constexpr int kPairSlots = 2 * kTilePx;

// Least edge key per unordered pair {a, b} of local components (a, b <
// kTilePx): open addressing on the pair, then a 64-bit atomic minimum.
// Returns the slot, or -1 if the table is full (the edge is then kept).
__device__ __forceinline__ int pair_min(int32_t *pk, unsigned long long *pv, int a, int b,
                                        uint64_t key) {
    const int pair = (a < b ? a : b) * kTilePx + (a < b ? b : a);
    int h = (int)(((uint32_t)pair * 2654435761u) >> 21) & (kPairSlots - 1);
    for (int it = 0; it < kPairSlots; ++it) {
        const int old = atomicCAS(&pk[h], -1, pair);
        if (old == -1 || old == pair) {
            if (pv[h] > key) atomicMin(&pv[h], (unsigned long long)key);
            return h;
        }
        h = (h + 1) & (kPairSlots - 1);
    }
    return -1;
}

__global__ __launch_bounds__(kLocalThreads) void k_local_msf(
    const float4 *__restrict__ img, LevelGeom g, const int32_t *__restrict__ plo,
    const int32_t *__restrict__ phi, int max_width, const int32_t *__restrict__ rank,
    int32_t *__restrict__ comp0,
    uint64_t *__restrict__ cw, uint64_t *__restrict__ best0, uint64_t *__restrict__ best1,
    int32_t *__restrict__ lmin, int32_t *__restrict__ croot, int32_t *__restrict__ mnroot,
    uint8_t *__restrict__ intree, uint64_t *__restrict__ E, int32_t *__restrict__ R,
    int32_t *__restrict__ ctr, int32_t *__restrict__ info) {
    __shared__ uint32_t kL[kTile], kU[kTile], kR[kTilePx], kD[kTilePx];
    __shared__ int32_t lab[kTilePx], hk[kTilePx];
    __shared__ unsigned long long best[kTilePx];
    __shared__ uint8_t tR[kTilePx], tD[kTilePx];  // tree edges taken, by owning pixel
    __shared__ int32_t pk[kPairSlots];               // component pair of a table slot
    __shared__ unsigned long long pv[kPairSlots];    // least (key, id) edge of the pair
    __shared__ int s_flag[2], s_nE, s_nR, s_bE, s_bR;
    const TileInfo t = tile_info(g, blockIdx.x);
    const float scale = ldexpf(1.0f, 2 * g.level);
    const int i = threadIdx.x;
    const int lx = i & (kTile - 1), ly = i >> 5;
    const bool valid = lx < t.tw && ly < t.th;
    const int64_t v = valid ? tile_pixel(t, i) : 0;
    if (i < kTile) {
        kL[i] = kNoKey;
        kU[i] = kNoKey;
    }
    if (i == 0) {
        s_nE = 0;
        s_nR = 0;
        s_bE = 0;
        s_bR = 0;
        s_flag[0] = 0;
        s_flag[1] = 0;
    }
    lab[i] = i;
    best[i] = kNoEdge;
    tR[i] = 0;
    tD[i] = 0;
    __syncthreads();
    // keys of the owned right / down edges (and of the edges entering from the
    // left / top neighbour tiles); an edge between different intervals is
    // absent.  Every load is issued first (clamped to the pixel itself where a
    // neighbour does not exist), then the edges are decided.
    uint32_t kr = kNoKey, kd = kNoKey;
    if (valid) {
        const int x = t.x0 + lx, y = t.y0 + ly;
        const bool hr = x + 1 < t.W, hd = y + 1 < t.H;
        const bool hl = lx == 0 && x > 0, hu = ly == 0 && y > 0;
        const int64_t vr = hr ? v + 1 : v, vd = hd ? v + t.W : v;
        const int64_t vl = hl ? v - 1 : v, vu = hu ? v - t.W : v;
        const float4 a = img[v], ar = img[vr], ad = img[vd], al = img[vl], au = img[vu];
        // random spanning tree: Kruskal's order is the edges' random ranks
        // (31 bits, so no rank is the absent-edge marker) instead of the colour key
        uint32_t qr = 0, qd = 0, ql = 0, qu = 0;
        if (rank) {
            qr = (uint32_t)rank[2 * v] & 0x7fffffffu;
            qd = (uint32_t)rank[2 * v + 1] & 0x7fffffffu;
            ql = (uint32_t)rank[2 * vl] & 0x7fffffffu;
            qu = (uint32_t)rank[2 * vu + 1] & 0x7fffffffu;
        }
        bool sr = true, sd = true, sl = true, su = true;
        if (plo) {
            const int lo = plo[v], hi = phi[v];
            const int lor = plo[vr], hir = phi[vr], lod = plo[vd], hid = phi[vd];
            const int lol = plo[vl], hil = phi[vl], lou = plo[vu], hiu = phi[vu];
            if (lo < 0 || hi < lo || hi > g.dmax[t.pair] || hi - lo + 1 > max_width)
                atomicAdd(&info[HDP_INFO_BAD_INTERVAL], 1);
            sr = lo == lor && hi == hir;
            sd = lo == lod && hi == hid;
            sl = lo == lol && hi == hil;
            su = lo == lou && hi == hiu;
        }
        if (hr && sr) kr = rank ? qr : edge_key(a, ar, scale);
        if (hd && sd) kd = rank ? qd : edge_key(a, ad, scale);
        if (hl && sl) kL[ly] = rank ? ql : edge_key(al, a, scale);
        if (hu && su) kU[lx] = rank ? qu : edge_key(au, a, scale);
    }
    kR[i] = kr;
    kD[i] = kd;
    const bool r_in = lx + 1 < t.tw, d_in = ly + 1 < t.th;
    __syncthreads();
    // (key, id) of the pixel's four edges; the left / up ones are the right /
    // down edges of the neighbour (or of the neighbour tile's pixel).  Ids are
    // tile-local, 2 * (halo row * kHalo + halo column) + direction of the
    // owning pixel: ordered as the global ids 2 * pixel + direction are, for
    // every edge this tile sees (both orders are row, column, direction).
    const uint32_t kl = lx == 0 ? kL[ly] : kR[i - 1], ku = ly == 0 ? kU[lx] : kD[i - kTile];
    const int hid = (ly + 1) * kHalo + lx + 1;
    const uint64_t er = kr != kNoKey ? key64(kr, 2 * hid) : kNoEdge;
    const uint64_t ed = kd != kNoKey ? key64(kd, 2 * hid + 1) : kNoEdge;
    const uint64_t el = valid && kl != kNoKey ? key64(kl, 2 * (hid - 1)) : kNoEdge;
    const uint64_t eu = valid && ku != kNoKey ? key64(ku, 2 * (hid - kHalo) + 1) : kNoEdge;
    const int lane = i & 63;
    // Boruvka rounds in LDS until no component hooks (each round with a hook
    // removes at least one component, so the loop ends).  A pixel's own label
    // and hook are written only by its thread and live in registers; the tree
    // edges are kept in LDS and stored once at the end, so that no barrier
    // waits on global stores.
    int myl = i;
    for (int iter = 0; iter < kTilePx; ++iter) {
        const int par = iter & 1;
        // every pixel offers its least edge to another component to its own
        // component; a wavefront whose offers all name one component makes
        // one atomic (late rounds, when components are large)
        int c = -1;
        uint64_t m = kNoEdge;
        if (valid) {
            c = myl;
            // the four neighbour labels, loaded together (an absent
            // neighbour reads the pixel's own slot)
            const int nr = lab[r_in ? i + 1 : i], nd = lab[d_in ? i + kTile : i];
            const int nl = lab[lx > 0 ? i - 1 : i], nu = lab[ly > 0 ? i - kTile : i];
            if (er != kNoEdge && (!r_in || nr != c)) m = er;
            if (ed != kNoEdge && (!d_in || nd != c)) m = ed < m ? ed : m;
            if (el != kNoEdge && (lx == 0 || nl != c)) m = el < m ? el : m;
            if (eu != kNoEdge && (ly == 0 || nu != c)) m = eu < m ? eu : m;
        }
        const bool has = m != kNoEdge;
        const uint64_t mh = __ballot(has);
        if (mh) {
            const int lead = __ffsll((unsigned long long)mh) - 1;
            const int c0 = __builtin_amdgcn_readlane(c, lead);
            if (__ballot(has && c != c0) == 0) {
                m = wave_min_u64(m);
                if (lane == lead && best[c0] > m) atomicMin(&best[c0], (unsigned long long)m);
            } else if (has && best[c] > m) {
                atomicMin(&best[c], (unsigned long long)m);
            }
        }
        __syncthreads();
        const uint64_t b = best[i];
        int hook = i;
        if (valid && myl == i && b != kNoEdge) {
            const uint32_t e = (uint32_t)b;
            const int o = (int)(e >> 1), oy = o / kHalo;
            const int px = o - oy * kHalo - 1, py = oy - 1;  // owning pixel, tile coordinates
            const int qx = px + (int)(~e & 1), qy = py + (int)(e & 1);
            const bool inside = px >= 0 && py >= 0 && qx < t.tw && qy < t.th;
            if (inside) {  // a least edge that leaves the tile waits for the global rounds
                int lp = py * kTile + px;
                int cp = lab[lp];
                int cq = lab[qy * kTile + qx];
                int other = cp == i ? cq : cp;
                if (!(best[other] == b && i < other)) {  // mutual choice: smaller index stays
                    hook = other;
                    if (e & 1) tD[lp] = 1;
                    else tR[lp] = 1;
                    s_flag[par] = 1;
                }
            }
        }
        __syncthreads();
        if (!s_flag[par]) break;  // best[] keeps this round's least edges
        best[i] = kNoEdge;
        if (i == 0) s_flag[par ^ 1] = 0;
        if (hook != i) {
            myl = hook;
            lab[i] = hook;
        }
        __syncthreads();
        // pointer jumping until every pixel names its root, without barriers
        // between the steps: a label only ever names an ancestor (a word its
        // owner has already advanced is just as valid) and roots stay roots
        // here, so a pixel is done once its label names itself; every step
        // moves a label to a strict ancestor, which bounds the loop
        for (int it = 0; it < kTilePx; ++it) {
            const int ll =
                __hip_atomic_load(&lab[myl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (ll == myl) break;
            myl = ll;
            __hip_atomic_store(&lab[i], ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
    }
    // smallest pixel id of every local component (hk reused); empty pair table
    hk[i] = 0x7fffffff;
    for (int h = i; h < kPairSlots; h += kLocalThreads) {
        pk[h] = -1;
        pv[h] = kNoEdge;
    }
    __syncthreads();
    if (valid) atomicMin(&hk[lab[i]], (int32_t)v);
    // Live edges: owned right / down edges not inside one component.  Of the
    // edges inside the tile joining the same two components only the least
    // (key, id) is kept: in the graph with the local components contracted the
    // others are the heavier of two parallel edges, never in the forest.
    const int c = lab[i];
    const int cr = r_in ? lab[i + 1] : -1, cd = d_in ? lab[i + kTile] : -1;
    bool live_r = valid && kr != kNoKey && cr != c;
    bool live_d = valid && kd != kNoKey && cd != c;
    const uint64_t gr = key64(kr, 2 * v), gd = key64(kd, 2 * v + 1);
    const int sr = live_r && cr >= 0 ? pair_min(pk, pv, c, cr, gr) : -1;
    const int sd = live_d && cd >= 0 ? pair_min(pk, pv, c, cd, gd) : -1;
    __syncthreads();
    if (sr >= 0 && pv[sr] != gr) live_r = false;
    if (sd >= 0 && pv[sd] != gd) live_d = false;
    // active components (with an incident edge left); reserve, then write
    const bool act = valid && c == i && best[i] != kNoEdge;
    const uint64_t mr = __ballot(live_r), md = __ballot(live_d), ma = __ballot(act);
    int wE = 0, wR = 0;
    if (lane == 0) {
        wE = atomicAdd(&s_nE, __popcll(mr) + __popcll(md));
        wR = atomicAdd(&s_nR, __popcll(ma));
    }
    __syncthreads();
    if (i == 0 && (s_nE | s_nR)) {  // both reservations in one 64-bit atomic
        static_assert(CTR_RALL == CTR_E + 1 && CTR_E % 2 == 0, "adjacent counters");
        const unsigned long long old =
            atomicAdd(reinterpret_cast<unsigned long long *>(&ctr[CTR_E]),
                      (unsigned long long)(uint32_t)s_nE | ((unsigned long long)s_nR << 32));
        s_bE = (int)(uint32_t)old;
        s_bR = (int)(old >> 32);
    }
    __syncthreads();
    wE = __shfl(wE, 0, 64) + s_bE;
    wR = __shfl(wR, 0, 64) + s_bR;
    const uint64_t lt = lanemask_lt();
    if (live_r) E[wE + __popcll(mr & lt)] = gr;
    if (live_d) E[wE + __popcll(mr) + __popcll(md & lt)] = gd;
    if (act) R[wR + __popcll(ma & lt)] = (int32_t)v;
    if (valid) {
        *reinterpret_cast<uint16_t *>(&intree[2 * v]) = (uint16_t)(tR[i] | (tD[i] << 8));
        comp0[v] = (int32_t)tile_pixel(t, c);
        if (c == i) {
            cw[v] = (uint64_t)(uint32_t)v;
            // least live edge of the component: the first global round's
            // minimum-edge step, already known here
            const uint64_t bl = best[i];
            if (bl != kNoEdge) {
                const int o = (int)((uint32_t)bl >> 1), oy = o / kHalo;
                const int64_t p = t.base + (int64_t)(t.y0 + oy - 1) * t.W + t.x0 + (o - oy * kHalo) - 1;
                best0[v] = key64((uint32_t)(bl >> 32), 2 * p + (int64_t)(bl & 1));
            } else {
                best0[v] = kNoEdge;
            }
            best1[v] = kNoEdge;
            lmin[v] = hk[i];
            // an active component keeps its slot in the active list here
            // until the roots step overwrites it (the tail numbers by it)
            croot[v] = act ? wR + __popcll(ma & lt) : -1;
            mnroot[v] = 0x7fffffff;
        }
    }
}

// --- 2. spanning forest: global rounds ---------------------------------------------
// A few full-grid rounds (minimum edge over the live-edge list, then hooking
// over the active components; dead edges are marked in place), then the edges
// still in play are compacted and one workgroup finishes in LDS.  Finds of
// round r's hooking step ignore round-r hooks, so every thread of that step
// sees the components as they were when it began.  Within a full-grid launch
// a thread may read a stale link; every link value ever stored is an ancestor,
// so a stale read only makes a find longer.

// Root of component x counting the hooks of rounds < cut.  kCoherent: read the
// links with device-coherent loads (needed when another wave of the same
// launch stored them and the reader must see it).
template <bool kCoherent>
__device__ __forceinline__ int find_comp(const uint64_t *cw, int x, int cut, int32_t *info) {
    // links form a forest; the bound only guards against a broken invariant
    for (int it = 0; it < (1 << 24); ++it) {
        uint64_t w = kCoherent ? ld_relaxed(&cw[x]) : cw[x];
        int y = (int)(uint32_t)w;
        int tag = (int)(w >> 32);
        if (y == x || (tag != 0 && tag - 1 >= cut)) return x;
        x = y;
    }
    info[HDP_INFO_ERROR] = 1;
    return x;
}

// Roots of components x and y counting the hooks of rounds < cut, the two
// link chains followed in lockstep (one batch of loads per step).
__device__ __forceinline__ void find_comp2(const uint64_t *cw, int &x, int &y, int cut,
                                           int32_t *info) {
    bool dx = false, dy = false;
    for (int it = 0; it < (1 << 24); ++it) {
        const uint64_t wx = dx ? 0 : cw[x], wy = dy ? 0 : cw[y];
        if (!dx) {
            const int nx = (int)(uint32_t)wx, tag = (int)(wx >> 32);
            if (nx == x || (tag != 0 && tag - 1 >= cut)) dx = true; else x = nx;
        }
        if (!dy) {
            const int ny = (int)(uint32_t)wy, tag = (int)(wy >> 32);
            if (ny == y || (tag != 0 && tag - 1 >= cut)) dy = true; else y = ny;
        }
        if (dx && dy) return;
    }
    info[HDP_INFO_ERROR] = 1;
}

__device__ __forceinline__ int other_end(const LevelGeom &g, uint32_t e) {
    int p = (int)(e >> 1);
    return (e & 1) ? p + g.W[pair_of(g, p)] : p + 1;
}

template <bool kCoherent>
__device__ __forceinline__ uint64_t ld_maybe(const uint64_t *p) {
    return kCoherent ? ld_relaxed(p) : *p;
}

// Current components of both ends of edge k (with path shortcuts).
template <bool kCoherent>
__device__ __forceinline__ void edge_comps(const LevelGeom &g, uint64_t k,
                                           const int32_t *__restrict__ comp0, uint64_t *cw, int *a,
                                           int *b, int32_t *info) {
    uint32_t e = (uint32_t)k;
    int p = (int)(e >> 1), q = other_end(g, e);
    int a0 = comp0[p], b0 = comp0[q];
    *a = find_comp<kCoherent>(cw, a0, 1 << 30, info);
    *b = find_comp<kCoherent>(cw, b0, 1 << 30, info);
    if (*a != a0) st_relaxed(&cw[a0], (uint64_t)(uint32_t)*a);  // shortcut (permanent link)
    if (*b != b0) st_relaxed(&cw[b0], (uint64_t)(uint32_t)*b);
}

__device__ __forceinline__ void offer_min(uint64_t *best, int x, uint64_t k, uint64_t seen) {
    if (seen > k) atomicMin((unsigned long long *)&best[x], (unsigned long long)k);
}

// kList: a round on the compacted list of live edges (the rounds after the
// compaction) instead of the whole list left by the tile-local phase.
template <bool kList>
__global__ __launch_bounds__(kBlock) void k_gbv_minedge(
    int round, const int32_t *__restrict__ flags, const int32_t *__restrict__ ctr, LevelGeom g,
    uint64_t *__restrict__ E, const int32_t *__restrict__ comp0, uint64_t *__restrict__ cw,
    uint64_t *__restrict__ best, int32_t *__restrict__ info) {
    // counters loaded together with the round's flag
    const int nLive = ctr[CTR_E], nE = kList ? ctr[CTR_ET] : nLive;
    const int more = round > 0 ? flags[FLAG_BV + round - 1] : 1;
    if (nLive <= kTE) return;  // small contracted graph: the tail alone
    if (more == 0) return;
    for (int i = (int)gtid(); i < nE; i += gridDim.x * kBlock) {
        uint64_t k = E[i];
        if (k == kNoEdge) continue;
        const uint32_t e = (uint32_t)k;
        const int a0 = comp0[e >> 1], b0 = comp0[other_end(g, e)];
        int a = a0, b = b0;
        find_comp2(cw, a, b, 1 << 30, info);
        if (a != a0) st_relaxed(&cw[a0], (uint64_t)(uint32_t)a);  // shortcut (permanent link)
        if (b != b0) st_relaxed(&cw[b0], (uint64_t)(uint32_t)b);
        if (a == b) {  // both ends in one component: never needed again
            E[i] = kNoEdge;
            continue;
        }
        const uint64_t ba = best[a], bb = best[b];
        offer_min(best, a, k, ba);
        offer_min(best, b, k, bb);
    }
}

__global__ __launch_bounds__(kBlock) void k_gbv_hook(
    int round, int32_t *__restrict__ flags, const int32_t *__restrict__ ctr, LevelGeom g,
    const int32_t *__restrict__ R, const int32_t *__restrict__ comp0, uint64_t *__restrict__ cw,
    const uint64_t *__restrict__ best, uint64_t *__restrict__ best_next,
    uint8_t *__restrict__ intree, int32_t *__restrict__ info) {
    const int nE = ctr[CTR_E], nR = ctr[CTR_RALL];  // loaded together with the flag
    const int more = round > 0 ? flags[FLAG_BV + round - 1] : 1;
    if (nE <= kTE) return;
    if (more == 0) return;
    bool hooked = false;
    for (int j = (int)gtid(); j < nR; j += gridDim.x * kBlock) {
        int x = R[j];
        const uint64_t wx = cw[x];
        const uint64_t b = best[x];
        if ((int)(uint32_t)wx != x) continue;  // hooked in an earlier round
        best_next[x] = kNoEdge;
        if (b == kNoEdge) continue;  // no edge left: its tree is complete
        uint32_t e = (uint32_t)b;
        int cp = comp0[e >> 1], cq = comp0[other_end(g, e)];
        find_comp2(cw, cp, cq, round, info);
        int other = cp == x ? cq : cp;
        if (best[other] == b && x < other) continue;  // mutual choice: the smaller id stays root
        st_relaxed(&cw[x], ((uint64_t)(round + 1) << 32) | (uint32_t)other);
        intree[e] = 1;
        hooked = true;
    }
    if (__ballot(hooked) && (threadIdx.x & 63) == 0) flags[FLAG_BV + round] = 1;
}

// edges still joining two components after the full-grid rounds
__global__ __launch_bounds__(kBlock) void k_gbv_compact(
    int K, const int32_t *__restrict__ flags, int32_t *__restrict__ ctr, LevelGeom g,
    const uint64_t *__restrict__ E, const int32_t *__restrict__ comp0, uint64_t *__restrict__ cw,
    uint64_t *__restrict__ Et, int32_t *__restrict__ info) {
    const int nE = ctr[CTR_E];
    const int more = K > 0 ? flags[FLAG_BV + K - 1] : 1;
    if (nE <= kTE || more == 0) return;  // tail alone (reads the live list) or done
    for (int i = (int)gtid(); i < nE; i += gridDim.x * kBlock) {
        uint64_t k = E[i];
        bool live = false;
        if (k != kNoEdge) {
            int a, b;
            edge_comps<false>(g, k, comp0, cw, &a, &b, info);
            live = a != b;
        }
        int pos = wave_append(live, &ctr[CTR_ET]);
        if (live) Et[pos] = k;
    }
}

// Hooking of a round on the compacted list, driven by the edges: a component
// hooks along the one live edge equal to its minimum (mutual choice: the
// smaller id stays the root), and the next round's minima of both ends are
// cleared (every component of the next round is an end of a live edge).  The
// components are those at the start of the round: links stored in this launch
// carry round + 1 and are not followed.
__global__ __launch_bounds__(kBlock) void k_gbv_lhook(
    int round, int32_t *__restrict__ flags, const int32_t *__restrict__ ctr, LevelGeom g,
    const uint64_t *__restrict__ Et, const int32_t *__restrict__ comp0, uint64_t *__restrict__ cw,
    const uint64_t *__restrict__ best, uint64_t *__restrict__ best_next,
    uint8_t *__restrict__ intree, int32_t *__restrict__ info) {
    const int nLive = ctr[CTR_E], nE = ctr[CTR_ET];  // loaded together with the flag
    const int more = flags[FLAG_BV + round - 1];
    if (nLive <= kTE || more == 0) return;
    bool hooked = false;
    for (int i = (int)gtid(); i < nE; i += gridDim.x * kBlock) {
        const uint64_t k = Et[i];
        if (k == kNoEdge) continue;
        const uint32_t e = (uint32_t)k;
        int a = comp0[e >> 1], b = comp0[other_end(g, e)];
        find_comp2(cw, a, b, round, info);
        if (a == b) continue;
        best_next[a] = kNoEdge;
        best_next[b] = kNoEdge;
        const uint64_t ba = best[a], bb = best[b];
        const uint64_t link = (uint64_t)(round + 1) << 32;
        if (ba == k && !(bb == k && a < b)) {
            st_relaxed(&cw[a], link | (uint32_t)b);
            intree[e] = 1;
            hooked = true;
        } else if (bb == k && !(ba == k && b < a)) {
            st_relaxed(&cw[b], link | (uint32_t)a);
            intree[e] = 1;
            hooked = true;
        }
    }
    if (__ballot(hooked) && (threadIdx.x & 63) == 0) flags[FLAG_BV + round] = 1;
}

// The remaining rounds in one workgroup.  With at most kTE edges and kTN
// components the contracted graph is loaded into LDS and finished there;
// otherwise the rounds run on the global arrays with device-coherent loads.
// After full-grid rounds the surviving components are renumbered through a
// hash table.  Without them (none launched, or all skipped because the graph
// has at most kTE edges) nothing has hooked yet: the live list itself is read
// (its edges join distinct active components), and when the graph fits LDS a
// component's dense number is its slot in the active list (kept in croot by
// the local phase).

__device__ __forceinline__ int hash_slot(int key) {
    return (int)(((uint32_t)key * 2654435761u) >> 20) & (kTH - 1);
}

__global__ __launch_bounds__(kLocalThreads) void k_gbv_tail(
    int K, int32_t *__restrict__ flags, const int32_t *__restrict__ ctr, LevelGeom g,
    uint64_t *__restrict__ E, uint64_t *__restrict__ Ec, const int32_t *__restrict__ comp0,
    uint64_t *__restrict__ cw, const int32_t *__restrict__ R, const int32_t *__restrict__ ridx,
    uint64_t *__restrict__ best0, uint64_t *__restrict__ best1, uint8_t *__restrict__ intree,
    int32_t *__restrict__ info) {
    static_assert(kTailEdgesPerThread * kLocalThreads == kTE, "edges per thread");
    __shared__ unsigned long long ek[kTE];
    __shared__ uint16_t ea[kTE], eb[kTE];
    __shared__ int32_t hkey[kTH];
    __shared__ uint16_t hval[kTH];
    __shared__ int32_t rid[kTN];
    __shared__ uint16_t lab[kTN], hk[kTN], bidx[kTN];
    __shared__ unsigned long long best[kTN];
    __shared__ int s_nodes, s_flag;
    // counters loaded together with the flag
    const int nLive = ctr[CTR_E], nComp = ctr[CTR_ET], nR = ctr[CTR_RALL];
    const int prev = K > 0 ? flags[FLAG_BV + K - 1] : 1;
    if (nLive > kTE && prev == 0) return;
    const int tid = threadIdx.x;
    const bool alone = K == 0 || nLive <= kTE;  // no full-grid round has run
    uint64_t *const Et = alone ? E : Ec;
    const int nE = alone ? nLive : nComp;
    const bool direct = alone && nR <= kTN;
    bool lds_mode = nE <= kTE;
    int ra[kTailEdgesPerThread], rb[kTailEdgesPerThread];  // endpoint components (pixel ids)
    uint64_t k0[kTailEdgesPerThread];
    if (direct) {
        if (tid == 0) s_nodes = nR;
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            const int i = tid + q * kLocalThreads;
            k0[q] = i < nE ? Et[i] : kNoEdge;
        }
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            ra[q] = rb[q] = -1;
            if (k0[q] == kNoEdge) continue;
            const uint32_t e = (uint32_t)k0[q];
            ra[q] = comp0[e >> 1];
            rb[q] = comp0[other_end(g, e)];
        }
        for (int j = tid; j < nR; j += kLocalThreads) rid[j] = R[j];
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            if (k0[q] == kNoEdge) continue;
            ek[tid + q * kLocalThreads] = k0[q];
        }
        __syncthreads();
    } else if (lds_mode) {
        for (int h = tid; h < kTH; h += kLocalThreads) hkey[h] = -1;
        if (tid == 0) s_nodes = 0;
        __syncthreads();
        // components of every edge (no link changes in this launch yet), into
        // the hash table of components.  A thread resolves its edges together:
        // one batch of loads per step of the link chains.
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            const int i = tid + q * kLocalThreads;
            k0[q] = i < nE ? Et[i] : kNoEdge;
        }
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            ra[q] = rb[q] = -1;
            if (k0[q] == kNoEdge) continue;
            const uint32_t e = (uint32_t)k0[q];
            ra[q] = comp0[e >> 1];
            rb[q] = comp0[other_end(g, e)];
        }
        for (int it = 0; it < (1 << 24); ++it) {  // links form a forest
            uint64_t wa[kTailEdgesPerThread], wb[kTailEdgesPerThread];
#pragma unroll
            for (int q = 0; q < kTailEdgesPerThread; ++q) {
                wa[q] = ra[q] >= 0 ? cw[ra[q]] : 0;
                wb[q] = rb[q] >= 0 ? cw[rb[q]] : 0;
            }
            bool more = false;
#pragma unroll
            for (int q = 0; q < kTailEdgesPerThread; ++q) {
                if (ra[q] < 0) continue;
                const int ya = (int)(uint32_t)wa[q], yb = (int)(uint32_t)wb[q];
                if (ya != ra[q]) { ra[q] = ya; more = true; }
                if (yb != rb[q]) { rb[q] = yb; more = true; }
            }
            if (!more) break;
        }
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            if (k0[q] == kNoEdge) continue;
            ek[tid + q * kLocalThreads] = k0[q];
            for (int c : {ra[q], rb[q]}) {
                int h = hash_slot(c);
                for (int it = 0; it < kTH; ++it) {
                    int old = atomicCAS(&hkey[h], -1, c);
                    if (old == -1 || old == c) break;
                    h = (h + 1) & (kTH - 1);
                }
            }
        }
        __syncthreads();
        // dense component numbers (a full table means more than kTN components)
        for (int h = tid; h < kTH; h += kLocalThreads) {
            int key = hkey[h];
            if (key < 0) continue;
            int idx = atomicAdd(&s_nodes, 1);
            hval[h] = (uint16_t)idx;
            if (idx < kTN) rid[idx] = key;
        }
        __syncthreads();
        lds_mode = s_nodes <= kTN;
    }
    if (lds_mode) {
        // Rounds in LDS.  Each thread keeps its edges (key, dense endpoints) in
        // registers and loads what a pass needs for all of them at once.
        const int nN = s_nodes;
        auto lookup = [&](int key) {
            int h = hash_slot(key);
            for (int it = 0; it < kTH && hkey[h] != key; ++it) h = (h + 1) & (kTH - 1);
            return hval[h];
        };
        uint64_t mk[kTailEdgesPerThread];
        int ma[kTailEdgesPerThread], mb[kTailEdgesPerThread];
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            const int i = tid + q * kLocalThreads;
            mk[q] = kNoEdge;
            ma[q] = mb[q] = 0;
            if (i >= nE) continue;
            mk[q] = k0[q];
            ma[q] = direct ? ridx[ra[q]] : lookup(ra[q]);
            mb[q] = direct ? ridx[rb[q]] : lookup(rb[q]);
        }
#pragma unroll
        for (int q = 0; q < kTailEdgesPerThread; ++q) {
            const int i = tid + q * kLocalThreads;
            if (i >= nE) continue;
            ea[i] = (uint16_t)ma[q];
            eb[i] = (uint16_t)mb[q];
        }
        // components j = tid + k * kLocalThreads belong to this thread, which
        // alone writes their label (kept in registers too)
        constexpr int kTailNodesPerThread = kTN / kLocalThreads;
        static_assert(kTailNodesPerThread * kLocalThreads == kTN, "nodes per thread");
        int ml[kTailNodesPerThread];
#pragma unroll
        for (int k = 0; k < kTailNodesPerThread; ++k) {
            const int j = tid + k * kLocalThreads;
            ml[k] = j;
            if (j >= nN) continue;
            lab[j] = (uint16_t)j;
            hk[j] = (uint16_t)j;
            best[j] = kNoEdge;
        }
        if (tid == 0) s_flag = 0;
        __syncthreads();
        for (int iter = 0; iter < kTN; ++iter) {
            // least live edge of every component (dead edges drop out for good)
            int ca[kTailEdgesPerThread], cb[kTailEdgesPerThread];
#pragma unroll
            for (int q = 0; q < kTailEdgesPerThread; ++q) {
                ca[q] = lab[ma[q]];
                cb[q] = lab[mb[q]];
            }
#pragma unroll
            for (int q = 0; q < kTailEdgesPerThread; ++q) {
                if (ca[q] == cb[q]) mk[q] = kNoEdge;
                if (mk[q] == kNoEdge) continue;
                if (best[ca[q]] > mk[q]) atomicMin(&best[ca[q]], (unsigned long long)mk[q]);
                if (best[cb[q]] > mk[q]) atomicMin(&best[cb[q]], (unsigned long long)mk[q]);
            }
            __syncthreads();
            // the edge that is each component's minimum
#pragma unroll
            for (int q = 0; q < kTailEdgesPerThread; ++q) {
                if (mk[q] == kNoEdge) continue;
                const uint16_t i = (uint16_t)(tid + q * kLocalThreads);
                if (best[ca[q]] == mk[q]) bidx[ca[q]] = i;
                if (best[cb[q]] == mk[q]) bidx[cb[q]] = i;
            }
            __syncthreads();
            // hooks (mutual choice: the smaller index stays the root); a hooked
            // component never becomes a root again, so its bidx keeps the edge
            bool hooked = false;
#pragma unroll
            for (int k = 0; k < kTailNodesPerThread; ++k) {
                const int j = tid + k * kLocalThreads;
                if (j >= nN || ml[k] != j) continue;
                const uint64_t bj = best[j];
                if (bj == kNoEdge) continue;
                const int i = bidx[j];
                const int xa = lab[ea[i]], xb = lab[eb[i]];
                const int other = xa == j ? xb : xa;
                if (best[other] == bj && j < other) continue;
                hk[j] = (uint16_t)other;
                hooked = true;
            }
            if (hooked) s_flag = iter + 1;
            __syncthreads();
            if (s_flag != iter + 1) break;
            if (tid == 0 && K + iter < 64) flags[FLAG_BV + K + iter] = 1;
#pragma unroll
            for (int k = 0; k < kTailNodesPerThread; ++k) {
                const int j = tid + k * kLocalThreads;
                if (j >= nN) continue;
                best[j] = kNoEdge;
                const int h = hk[j];
                if (h != j) {
                    ml[k] = h;
                    lab[j] = (uint16_t)h;
                    hk[j] = (uint16_t)j;
                }
            }
            __syncthreads();
            // pointer jumping until every component names its root, without
            // barriers between the steps (labels only move to ancestors, roots
            // stay roots: a node is done once its label names itself)
            volatile uint16_t *vlab = lab;
            uint32_t open = 0;
#pragma unroll
            for (int k = 0; k < kTailNodesPerThread; ++k)
                if (tid + k * kLocalThreads < nN) open |= 1u << k;
            for (int it = 0; open && it < kTN; ++it) {
                int ll[kTailNodesPerThread];
#pragma unroll
                for (int k = 0; k < kTailNodesPerThread; ++k)
                    ll[k] = ((open >> k) & 1) ? vlab[ml[k]] : ml[k];
#pragma unroll
                for (int k = 0; k < kTailNodesPerThread; ++k) {
                    if (!((open >> k) & 1)) continue;
                    if (ll[k] == ml[k]) {
                        open &= ~(1u << k);
                        continue;
                    }
                    ml[k] = ll[k];
                    vlab[tid + k * kLocalThreads] = (uint16_t)ll[k];
                }
            }
            __syncthreads();
        }
        // tree edges and permanent links of every merged component
        for (int j = tid; j < nN; j += kLocalThreads) {
            int r = lab[j];
            if (r == j) continue;
            intree[(uint32_t)ek[bidx[j]]] = 1;
            cw[rid[j]] = (uint64_t)(uint32_t)rid[r];
        }
        return;
    }
    // large case: rounds on the global arrays, hooking driven by the edges
    // (each component hooks along the one edge equal to its minimum)
    for (int r = K; r < 64; ++r) {
        uint64_t *cur = (r & 1) ? best1 : best0, *nxt = (r & 1) ? best0 : best1;
        for (int i = tid; i < nE; i += kLocalThreads) {
            uint64_t k = ld_relaxed(&Et[i]);
            if (k == kNoEdge) continue;
            int a, b;
            edge_comps<true>(g, k, comp0, cw, &a, &b, info);
            if (a == b) {
                st_relaxed(&Et[i], kNoEdge);
                continue;
            }
            offer_min(cur, a, k, ld_relaxed(&cur[a]));
            offer_min(cur, b, k, ld_relaxed(&cur[b]));
        }
        if (tid == 0) s_flag = 0;
        wg_sync();
        bool hooked = false;
        for (int i = tid; i < nE; i += kLocalThreads) {
            uint64_t k = ld_relaxed(&Et[i]);
            if (k == kNoEdge) continue;
            uint32_t e = (uint32_t)k;
            int a = find_comp<true>(cw, comp0[e >> 1], r, info);
            int b = find_comp<true>(cw, comp0[other_end(g, e)], r, info);
            st_relaxed(&nxt[a], kNoEdge);
            st_relaxed(&nxt[b], kNoEdge);
            for (int side = 0; side < 2; ++side) {
                int x = side ? b : a, other = side ? a : b;
                if (ld_relaxed(&cur[x]) != k) continue;
                if (ld_relaxed(&cur[other]) == k && x < other) continue;
                st_relaxed(&cw[x], ((uint64_t)(r + 1) << 32) | (uint32_t)other);
                intree[e] = 1;
                hooked = true;
            }
        }
        if (hooked) s_flag = 1;
        wg_sync();
        int any = s_flag;
        if (!any) break;
        if (tid == 0) flags[FLAG_BV + r] = 1;
        __syncthreads();  // every thread has read s_flag before it is cleared
    }
}

// --- 3. roots: smallest pixel id of every tree -------------------------------------

__global__ __launch_bounds__(kBlock) void k_gbv_final(
    const int32_t *__restrict__ ctr, const int32_t *__restrict__ R,
    const uint64_t *__restrict__ cw, const int32_t *__restrict__ lmin,
    int32_t *__restrict__ croot, int32_t *__restrict__ mnroot, int32_t *__restrict__ info) {
    const int nR = ctr[CTR_RALL];
    // uniform trip count, so every lane takes part in the wavefront reductions
    for (int base = blockIdx.x * kBlock; base < nR; base += gridDim.x * kBlock) {
        const int j = base + (int)threadIdx.x;
        const bool valid = j < nR;
        int r = -1, m = 0x7fffffff;
        if (valid) {
            int x = R[j];
            r = find_comp<false>(cw, x, 1 << 30, info);
            croot[x] = r;
            m = lmin[x];
        }
        const uint64_t mv = __ballot(valid);
        if (mv == 0) continue;
        const int lead = __ffsll((unsigned long long)mv) - 1;
        const int r0 = __shfl(r, lead, 64);
        if (__ballot(valid && r != r0) == 0) {
            // one tree in this wavefront (the common case): one atomic
            for (int off = 32; off > 0; off >>= 1) {
                int o = __shfl_xor(m, off, 64);
                m = o < m ? o : m;
            }
            if ((int)(threadIdx.x & 63) == lead && mnroot[r0] > m) atomicMin(&mnroot[r0], m);
        } else if (valid && mnroot[r] > m) {
            atomicMin(&mnroot[r], m);
        }
    }
}

// tree id (root pixel) of every pixel and its tree-edge bits: 1 right, 2 down,
// 4 left, 8 up; bit 16 marks the root
constexpr uint8_t kRootBit = 16;

__global__ void k_set_tree(const int32_t *__restrict__ comp0, const int32_t *__restrict__ croot,
                           const int32_t *__restrict__ lmin, const int32_t *__restrict__ mnroot,
                           const uint8_t *__restrict__ intree, LevelGeom g,
                           int32_t *__restrict__ tree, uint8_t *__restrict__ adj,
                           int32_t *__restrict__ info) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    const PixelPos p = pixel_pos(g, (int)v);
    // the four edge bits load together with the component chain
    const uint8_t er = intree[2 * v], ed = intree[2 * v + 1];
    const uint8_t el = intree[p.x > 0 ? 2 * (v - 1) : 2 * v];
    const uint8_t eu = intree[p.y > 0 ? 2 * (v - p.W) + 1 : 2 * v];
    int x = comp0[v];
    int c = croot[x];
    int t = c >= 0 ? mnroot[c] : lmin[x];
    tree[v] = t;
    uint8_t a = 0;
    if (er) a |= 1;
    if (ed) a |= 2;
    if (p.x > 0 && el) a |= 4;
    if (p.y > 0 && eu) a |= 8;
    if (t == v) a |= kRootBit;
    adj[v] = a;
}

// --- literal disparity forest (outside the exact regime) -------------------------
// Section 3.2 as written: Kruskal over the grid edges in ascending (weight,
// edge id) with Rule 2 (union-find), DT-Rule 1 (eq. cri1: skip an edge whose
// two pixel intervals are disjoint) and DT-Rule 2 (eq. DTrules on the current
// tree intervals, tested exactly as beta_den * |n| >= beta_num * |u|; a merge
// gives the tree the union of the two intervals).  Outside the regime of
// equal intervals the result depends on the order, so the edges are sorted by
// (key, id) and one workgroup takes them in that order.

// Keys and the DT-Rule 1 filter of the two edges a pixel owns (sentinel:
// absent or filtered, sorted last), and the start state of the union-find.
__global__ void k_seq_edges(const float4 *__restrict__ img, LevelGeom g,
                            const int32_t *__restrict__ plo, const int32_t *__restrict__ phi,
                            const int32_t *__restrict__ rank, uint32_t sentinel,
                            uint32_t *__restrict__ ekey,
                            int32_t *__restrict__ uf, int32_t *__restrict__ usz,
                            int32_t *__restrict__ tlo, int32_t *__restrict__ thi,
                            int32_t *__restrict__ croot, int32_t *__restrict__ lmin,
                            uint8_t *__restrict__ intree, int32_t *__restrict__ info) {
    const int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    const PixelPos p = pixel_pos(g, (int)v);
    const bool hr = p.x + 1 < p.W, hd = p.y + 1 < p.H;
    const int64_t vr = hr ? v + 1 : v, vd = hd ? v + p.W : v;
    const float4 a = img[v], ar = img[vr], ad = img[vd];
    const int dm = g.dmax[p.pair];
    int l = plo[v], h = phi[v];
    const int lr = plo[vr], hrr = phi[vr], ld = plo[vd], hdd = phi[vd];
    const float scale = ldexpf(1.0f, 2 * g.level);
    // an interval that is empty or leaves [0, dmax] makes the forest invalid
    if (l < 0 || h > dm || l > h) atomicAdd(&info[HDP_INFO_BAD_INTERVAL], 1);
    const bool kr = hr && (l > lr ? l : lr) <= (h < hrr ? h : hrr);
    const bool kd = hd && (l > ld ? l : ld) <= (h < hdd ? h : hdd);
    // random spanning tree: the edges' random ranks (31 bits) order them instead
    const uint32_t qr = rank ? (uint32_t)rank[2 * v] & 0x7fffffffu : edge_key(a, ar, scale);
    const uint32_t qd = rank ? (uint32_t)rank[2 * v + 1] & 0x7fffffffu : edge_key(a, ad, scale);
    ekey[2 * v] = kr ? qr : sentinel;
    ekey[2 * v + 1] = kd ? qd : sentinel;
    l = l < 0 ? 0 : (l > dm ? dm : l);
    h = h < l ? l : (h > dm ? dm : h);
    uf[v] = (int32_t)v;
    usz[v] = 1;
    tlo[v] = l;
    thi[v] = h;
    croot[v] = -1;
    lmin[v] = 0x7fffffff;
    intree[2 * v] = 0;
    intree[2 * v + 1] = 0;
}

// digit of an edge's key for the stable counting sort of the edge ids
struct EdgeDigit {
    const uint32_t *key;
    int shift;
    __device__ int operator()(int64_t, int32_t e) const { return (key[e] >> shift) & 255; }
};

constexpr int kSeqThreads = 256;
constexpr int kSeqChunk = 2048;  // edges staged in LDS per step

__device__ __forceinline__ int32_t uf_root_ro(const int32_t *uf, int32_t v) {
    int32_t u = uf[v];
    while (u != v) {
        v = u;
        u = uf[v];
    }
    return v;
}

// The sequential process: the workgroup stages the next kSeqChunk edges of
// the sorted list in LDS with the roots of both ends as the chunk starts
// (found in parallel; roots only ever merge, so ends that share a root then
// are certainly a Rule 2 skip, and a root then is an ancestor of the root
// now), then one thread takes the edges in order and decides each exactly as
// in the definition above.
__global__ __launch_bounds__(kSeqThreads) void k_seq_kruskal(
    const int32_t *__restrict__ sorted, const uint32_t *__restrict__ ekey, int64_t m,
    uint32_t sentinel, LevelGeom g, int beta_num, int beta_den, int32_t *__restrict__ uf,
    int32_t *__restrict__ usz, int32_t *__restrict__ tlo, int32_t *__restrict__ thi,
    uint8_t *__restrict__ intree) {
    __shared__ int32_t se[kSeqChunk], sp[kSeqChunk], sq[kSeqChunk];
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    if (tid == 0) s_stop = 0;
    for (int64_t base = 0; base < m; base += kSeqChunk) {
        __syncthreads();
        if (s_stop) break;
        for (int j = tid; j < kSeqChunk; j += kSeqThreads) {
            const int64_t i = base + j;
            int32_t e = -1, hp = 0, hq = 0;
            if (i < m) {
                e = sorted[i];
                if (ekey[e] == sentinel) {
                    e = -1;  // absent or filtered: every later edge is too
                } else {
                    const int32_t pv = e >> 1;
                    const int32_t q = (e & 1) ? pv + g.W[pair_of(g, pv)] : pv + 1;
                    hp = uf_root_ro(uf, pv);
                    hq = uf_root_ro(uf, q);
                }
            }
            se[j] = e;
            sp[j] = hp;
            sq[j] = hq;
        }
        __syncthreads();
        if (tid == 0) {
            for (int j = 0; j < kSeqChunk; ++j) {
                const int32_t e = se[j];
                if (e < 0) {
                    s_stop = 1;
                    break;
                }
                int32_t rp = sp[j], rq = sq[j];
                if (rp == rq) continue;  // Rule 2 (one tree since the chunk began)
                // the roots now: both chains (merges of this chunk) walked together
                for (;;) {
                    const int32_t up = uf[rp], uq = uf[rq];
                    if (up == rp && uq == rq) break;
                    rp = up;
                    rq = uq;
                }
                if (rp == rq) continue;  // Rule 2
                // DT-Rule 2 on the current tree intervals
                const int32_t lp = tlo[rp], hp = thi[rp], lq = tlo[rq], hq = thi[rq];
                const int32_t zp = usz[rp], zq = usz[rq];
                const int32_t ilo = lp > lq ? lp : lq, ihi = hp < hq ? hp : hq;
                const int64_t inter = ihi >= ilo ? (int64_t)(ihi - ilo + 1) : 0;
                const int64_t uni = (int64_t)(hp - lp + 1) + (hq - lq + 1) - inter;
                if ((int64_t)beta_den * inter < (int64_t)beta_num * uni) continue;
                // merge (union by size); the tree takes the union of the intervals
                if (zp < zq) {
                    const int32_t t = rp;
                    rp = rq;
                    rq = t;
                }
                uf[rq] = rp;
                usz[rp] = zp + zq;
                tlo[rp] = lp < lq ? lp : lq;
                thi[rp] = hp > hq ? hp : hq;
                intree[e] = 1;
            }
        }
    }
}

// Per pixel: its tree (union-find root), the tree's smallest pixel and the
// tree's interval; trees wider than the row width are counted as bad.
__global__ void k_seq_roots(const int32_t *__restrict__ uf, const int32_t *__restrict__ tlo,
                            const int32_t *__restrict__ thi, int64_t n, int width,
                            int32_t *__restrict__ comp0, int32_t *__restrict__ lmin,
                            int32_t *__restrict__ plo2, int32_t *__restrict__ phi2,
                            int32_t *__restrict__ info) {
    const int64_t v = gtid();
    if (v >= n) return;
    int32_t r = (int32_t)v;
    while (uf[r] != r) r = uf[r];
    comp0[v] = r;
    atomicMin(&lmin[r], (int32_t)v);
    const int32_t l = tlo[r], h = thi[r];
    plo2[v] = l;
    phi2[v] = h;
    if (h - l + 1 > width) atomicAdd(&info[HDP_INFO_BAD_INTERVAL], 1);
}

// --- 4. Euler tour ranking ---------------------------------------------------------
// Slot 4v+d = directed tree edge from v in direction d (0 right, 1 down, 2 left,
// 3 up); its successor turns to the next tree edge of the far pixel, and the
// tour of a tree ends at the slot that would return to the root's first edge.
// Rank = hops to the end of the tour.  Each tile first ranks, in LDS, the runs
// of its slots whose successors stay in the tile; a run ends at an exit (the
// successor lies in another tile) or at the tour's end.  The run ends form a
// short contracted list that pointer jumping ranks globally:
//   lw[s]  = (index of the end of s's run) << 32 | hops from s to that end
//   pr[i]  = (next run end) << 32 | hops, jumped until next = -1.

__device__ __forceinline__ int64_t nbr(int64_t v, int d, int W) {
    return d == 0 ? v + 1 : d == 1 ? v + W : d == 2 ? v - 1 : v - W;
}

__device__ __forceinline__ int first_dir(uint8_t a) { return __ffs((int)(a & 15)) - 1; }

// direction of the tour step after arriving through direction d at a pixel with edge bits aw
__device__ __forceinline__ int turn(uint8_t aw, int d) {
    int rd = d ^ 2, d2 = rd;
    for (int k = 1; k <= 4; ++k) {
        d2 = (rd + k) & 3;
        if ((aw >> d2) & 1) break;
    }
    return d2;
}

constexpr uint32_t kTourEnd = 0xFFFFFFFFu;
// The tile-local tour ranking runs 512 threads per tile (eight slots each):
// four tiles fit a compute unit at once instead of two.
constexpr int kTourThreads = 512;
constexpr int kTourSlots = 4 * kTilePx / kTourThreads;

__global__ __launch_bounds__(kTourThreads) void k_tour_local(
    LevelGeom g, const uint8_t *__restrict__ adj, uint64_t *__restrict__ lw,
    uint32_t *__restrict__ C, int32_t *__restrict__ ctr, int32_t *__restrict__ info) {
    __shared__ uint8_t sadj[kHalo * kHalo];
    __shared__ uint32_t P[4 * kTilePx];
    __shared__ int32_t tix[4 * kTilePx];
    __shared__ int s_n, s_base;
    const TileInfo t = tile_info(g, blockIdx.x);
    const int tid = threadIdx.x;
    for (int h = tid; h < kHalo * kHalo; h += kTourThreads) {
        int x = t.x0 + (h % kHalo) - 1, y = t.y0 + (h / kHalo) - 1;
        bool in = x >= 0 && x < t.W && y >= 0 && y < t.H;
        sadj[h] = in ? adj[t.base + (int64_t)y * t.W + x] : 0;
    }
    if (tid == 0) s_n = 0;
    __syncthreads();
    // slot ls = 4 * (ly * kTile + lx) + d; P = next << 16 | hops (run end:
    // next = self; a run has fewer than 4 * kTilePx hops)
    constexpr uint32_t kInvalid = ~0u;
    // Only the owning thread writes a slot, so each thread keeps its slots in
    // registers; a pointer-jumping round is one batch of independent loads.
    uint32_t own[kTourSlots];
    uint32_t live = 0;
    for (int k = 0; k < kTourSlots; ++k) {
        int ls = tid + k * kTourThreads;
        int i = ls >> 2, d = ls & 3;
        int lx = i & (kTile - 1), ly = i >> 5;
        uint32_t w = kInvalid;
        if (lx < t.tw && ly < t.th && ((sadj[(ly + 1) * kHalo + lx + 1] >> d) & 1)) {
            int wx = lx + (d == 0) - (d == 2), wy = ly + (d == 1) - (d == 3);
            uint8_t aw = sadj[(wy + 1) * kHalo + wx + 1];
            int d2 = turn(aw, d);
            bool end = (aw & kRootBit) && d2 == first_dir(aw);
            bool inside = wx >= 0 && wx < t.tw && wy >= 0 && wy < t.th;
            if (end || !inside) {
                w = (uint32_t)ls << 16;
            } else {
                w = ((uint32_t)(4 * (wy * kTile + wx) + d2) << 16) | 1u;
                live |= 1u << k;
            }
        }
        own[k] = w;
        P[ls] = w;
    }
    __syncthreads();
    // pointer jumping inside the tile, without barriers between the steps:
    // a slot word is written by its owner only and always names a later slot
    // of its run with the hops to it, so a word that its owner has already
    // advanced in this pass is just as valid (the reader gets there sooner).
    // A thread stops once its slots point at their run ends; every step
    // advances a slot by at least one hop, which bounds the loop.
    for (int step = 0; live && step <= 4 * kTilePx; ++step) {
        uint32_t nxt[kTourSlots];
        for (int k = 0; k < kTourSlots; ++k)
            nxt[k] = ((live >> k) & 1) ? __hip_atomic_load(&P[own[k] >> 16], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP)
                                       : 0u;
        for (int k = 0; k < kTourSlots; ++k) {
            if (!((live >> k) & 1)) continue;
            uint32_t nx = own[k] >> 16, nn = nxt[k] >> 16;
            if (nn == nx) {  // next is its run's end: done
                live &= ~(1u << k);
                continue;
            }
            own[k] = (nn << 16) | ((own[k] & 0xFFFFu) + (nxt[k] & 0xFFFFu));
            __hip_atomic_store(&P[tid + k * kTourThreads], own[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    if (live) info[HDP_INFO_ERROR] = 5;
    __syncthreads();
    // number the run ends (one LDS atomic per wavefront and slot group)
    int wofs[kTourSlots];
    uint64_t wm[kTourSlots];
    const int lane = tid & 63;
    for (int k = 0; k < kTourSlots; ++k) {
        int ls = tid + k * kTourThreads;
        bool term = own[k] != kInvalid && (int)(own[k] >> 16) == ls;
        wm[k] = __ballot(term);
        wofs[k] = 0;
        if (lane == 0 && wm[k]) wofs[k] = atomicAdd(&s_n, __popcll(wm[k]));
    }
    __syncthreads();
    if (tid == 0) s_base = s_n ? atomicAdd(&ctr[CTR_RUNS], s_n) : 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (int k = 0; k < kTourSlots; ++k) {
        int ls = tid + k * kTourThreads;
        int base = __shfl(wofs[k], 0, 64) + s_base;
        if (!((wm[k] >> lane) & 1)) continue;
        int idx = base + __popcll(wm[k] & lt);
        tix[ls] = idx;
        int i = ls >> 2, d = ls & 3;
        int lx = i & (kTile - 1), ly = i >> 5;
        int wx = lx + (d == 0) - (d == 2), wy = ly + (d == 1) - (d == 3);
        uint8_t aw = sadj[(wy + 1) * kHalo + wx + 1];
        int d2 = turn(aw, d);
        bool end = (aw & kRootBit) && d2 == first_dir(aw);
        int64_t wg = t.base + (int64_t)(t.y0 + wy) * t.W + t.x0 + wx;
        C[idx] = end ? kTourEnd : (uint32_t)(4 * wg + d2);
    }
    __syncthreads();
    for (int k = 0; k < kTourSlots; ++k) {
        int ls = tid + k * kTourThreads;
        uint32_t a = own[k];
        if (a == kInvalid) continue;
        int64_t v = tile_pixel(t, ls >> 2);
        lw[4 * v + (ls & 3)] = ((uint64_t)(uint32_t)tix[a >> 16] << 32) | (a & 0xFFFFu);
    }
}

// contracted list: run end i -> the end of the run its successor starts
__global__ __launch_bounds__(kBlock) void k_tour_link(const int32_t *__restrict__ ctr,
                                                      const uint32_t *__restrict__ C,
                                                      const uint64_t *__restrict__ lw,
                                                      uint64_t *__restrict__ pr) {
    const int nC = ctr[CTR_RUNS];
    for (int i = (int)gtid(); i < nC; i += gridDim.x * kBlock) {
        uint32_t s2 = C[i];
        if (s2 == kTourEnd) {
            pr[i] = (uint64_t)0xFFFFFFFFu << 32;
        } else {
            uint64_t w = lw[s2];
            pr[i] = (w & 0xFFFFFFFF00000000ull) | (uint32_t)((uint32_t)w + 1u);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_rank_round(int round, int32_t *__restrict__ flags,
                                                       const int32_t *__restrict__ ctr,
                                                       uint64_t *__restrict__ pr) {
    const int nC = ctr[CTR_RUNS];  // loaded together with the round's flag
    const int prev = round > 0 ? flags[FLAG_RANK + round - 1] : 1;
    if (nC <= kTA) return;  // short lists: the one-workgroup tail alone
    if (prev == 0) return;
    // Several jumps per launch, each published at once: an entry may read a
    // successor that has already jumped further in this launch, which only
    // shortens the way (every word is a valid "successor at that distance").
    bool more = false;
    for (int s = (int)gtid(); s < nC; s += gridDim.x * kBlock) {
        uint64_t P = ld_relaxed(&pr[s]);
        for (int j = 0; j < kRankJumps; ++j) {
            const int32_t nx = (int32_t)(P >> 32);
            if (nx < 0) break;
            const uint64_t Q = ld_relaxed(&pr[nx]);
            P = (Q & 0xFFFFFFFF00000000ull) | (uint32_t)((uint32_t)P + (uint32_t)Q);
            st_relaxed(&pr[s], P);
        }
        more |= (int32_t)(P >> 32) >= 0;
    }
    if (__ballot(more) && (threadIdx.x & 63) == 0) flags[FLAG_RANK + round] = 1;
}

__global__ __launch_bounds__(kBlock) void k_rank_compact(int K, const int32_t *__restrict__ flags,
                                                         int32_t *__restrict__ ctr,
                                                         const uint64_t *__restrict__ pr,
                                                         int32_t *__restrict__ At) {
    const int nC = ctr[CTR_RUNS];  // loaded together with the last round's flag
    const int prev = K > 0 ? flags[FLAG_RANK + K - 1] : 1;
    if (nC > kTA && prev == 0) return;
    for (int s = (int)gtid(); s < nC; s += gridDim.x * kBlock) {
        bool open = (int32_t)(pr[s] >> 32) >= 0;
        int pos = wave_append(open, &ctr[CTR_AT]);
        if (open) At[pos] = s;
    }
}

// The unfinished entries in one workgroup: renumbered into LDS (entries that
// point at a finished entry absorb its rank) and jumped there; a larger set
// is jumped on the global array with device-coherent loads.  A list short
// enough that no full-grid round ran is jumped in LDS as it stands (entry j
// at LDS slot j, no compaction or renumbering).
__global__ __launch_bounds__(kLocalThreads) void k_rank_tail(
    int K, int32_t *__restrict__ flags, const int32_t *__restrict__ ctr,
    const int32_t *__restrict__ At, int32_t *__restrict__ slot, uint64_t *__restrict__ pr,
    int32_t *__restrict__ info) {
    __shared__ unsigned long long L[kTA];
    __shared__ int s_more;
    const int nRuns = ctr[CTR_RUNS], nA = ctr[CTR_AT];  // loaded together with the flag
    const int prev = K > 0 ? flags[FLAG_RANK + K - 1] : 1;
    if (nRuns > kTA && prev == 0) return;
    const int tid = threadIdx.x;
    if (nRuns <= kTA) {
        // Each thread jumps its entries (kept in registers) without barriers
        // between the steps: an entry word is written by its owner only and
        // is always a valid successor with the hops to it.
        constexpr int kPer = kTA / kLocalThreads;
        unsigned long long own[kPer];
        uint32_t live = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kLocalThreads;
            own[q] = j < nRuns ? pr[j] : (0xFFFFFFFFull << 32);
            if ((int32_t)(own[q] >> 32) >= 0) live |= 1u << q;
            if (j < nRuns) L[j] = own[q];
        }
        // (the vote is also the barrier after the LDS fill)
        const int any_open = __syncthreads_or(live != 0);
        if (tid == 0 && any_open) flags[FLAG_RANK + K] = 1;
        for (int step = 0; live && step <= kTA; ++step) {
            unsigned long long nb[kPer];
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                nb[q] = ((live >> q) & 1) ? __hip_atomic_load(&L[(int32_t)(own[q] >> 32)],
                                                              __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_WORKGROUP)
                                          : 0ull;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                if (!((live >> q) & 1)) continue;
                own[q] = (nb[q] & 0xFFFFFFFF00000000ull) | (uint32_t)((uint32_t)own[q] + (uint32_t)nb[q]);
                __hip_atomic_store(&L[tid + q * kLocalThreads], own[q], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                if ((int32_t)(nb[q] >> 32) < 0) live &= ~(1u << q);
            }
        }
        if (live) info[HDP_INFO_ERROR] = 6;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kLocalThreads;
            if (j < nRuns) pr[j] = (0xFFFFFFFFull << 32) | (uint32_t)own[q];
        }
        return;
    }
    if (nA <= kTA) {
        for (int j = tid; j < nA; j += kLocalThreads) slot[At[j]] = j;
        wg_sync();
        for (int j = tid; j < nA; j += kLocalThreads) {
            uint64_t P = pr[At[j]];
            int nx = (int32_t)(P >> 32);
            uint64_t Q = pr[nx];
            if ((int32_t)(Q >> 32) < 0)
                L[j] = (0xFFFFFFFFull << 32) | (uint32_t)((uint32_t)P + (uint32_t)Q);
            else
                L[j] = ((uint64_t)(uint32_t)ld_relaxed(&slot[nx]) << 32) | (uint32_t)P;
        }
        for (int r = K; r < 64; ++r) {
            if (tid == 0) s_more = 0;
            __syncthreads();
            bool more = false;
            for (int j = tid; j < nA; j += kLocalThreads) {
                unsigned long long a = L[j];
                int nx = (int32_t)(a >> 32);
                if (nx < 0) continue;
                unsigned long long b = L[nx];
                L[j] = (b & 0xFFFFFFFF00000000ull) | (uint32_t)((uint32_t)a + (uint32_t)b);
                more |= (int32_t)(b >> 32) >= 0;
            }
            if (more) s_more = 1;
            __syncthreads();
            int any = s_more;
            __syncthreads();  // every thread has read s_more before it is cleared
            if (!any) break;
            if (tid == 0) flags[FLAG_RANK + r] = 1;
        }
        for (int j = tid; j < nA; j += kLocalThreads)
            pr[At[j]] = (0xFFFFFFFFull << 32) | (uint32_t)L[j];
        return;
    }
    for (int r = K; r < 64; ++r) {
        if (tid == 0) s_more = 0;
        wg_sync();
        bool more = false;
        for (int j = tid; j < nA; j += kLocalThreads) {
            int s = At[j];
            uint64_t P = ld_relaxed(&pr[s]);
            int32_t nx = (int32_t)(P >> 32);
            if (nx < 0) continue;
            uint64_t Q = ld_relaxed(&pr[nx]);
            int32_t nn = (int32_t)(Q >> 32);
            st_relaxed(&pr[s],
                       ((uint64_t)(uint32_t)nn << 32) | (uint32_t)((uint32_t)P + (uint32_t)Q));
            more |= nn >= 0;
        }
        if (more) s_more = 1;
        wg_sync();
        int any = s_more;
        if (!any) return;
        if (tid == 0) flags[FLAG_RANK + r] = 1;
        __syncthreads();  // every thread has read s_more before it is cleared
    }
    if (tid == 0) info[HDP_INFO_ERROR] = 6;
}

struct Ranks {
    const uint64_t *lw, *pr;
    __device__ __forceinline__ uint32_t operator()(int64_t s) const {
        uint64_t w = lw[s];
        return (uint32_t)w + (uint32_t)pr[w >> 32];
    }
};

// Node code of a pixel, packed so that the row-order kernels gather one 8-byte
// record (code, edge weight) per row: bits 0-4 tree-edge bits and root bit,
// 5-6 direction of the parent, 7 has a heavy child, 8-9 its direction,
// 16-23 interval low label, 24-31 interval high label (labels are below 256).
constexpr uint32_t kHasHeavy = 1u << 7;
__device__ __forceinline__ int code_pdir(uint32_t c) { return (c & kRootBit) ? -1 : (int)(c >> 5) & 3; }
__device__ __forceinline__ int code_hdir(uint32_t c) { return (c & kHasHeavy) ? (int)(c >> 8) & 3 : -1; }

// Per pixel (all writes coalesced): its parent (the tree neighbour whose edge
// toward it comes first on the tour), the weight of the edge to the parent
// (recomputed from the image with the key formula), its heavy child, the tree
// interval, the node record, and for a root its node count and the root data
// (tour length and node count, packed for one scan).
__device__ __forceinline__ uint64_t parent_of_pixel(
    int64_t v, const LevelGeom &g, const float4 *__restrict__ img, Ranks rank_of,
    const uint8_t *__restrict__ adj, const int32_t *__restrict__ plo,
    const int32_t *__restrict__ phi, int max_width, int32_t *__restrict__ parent,
    int32_t *__restrict__ size, float *__restrict__ wgt, uint64_t *__restrict__ rootval,
    int32_t *__restrict__ lo, int32_t *__restrict__ hi, uint2 *__restrict__ nrec) {
    const int pair = pair_of(g, (int)v);
    const int W = g.W[pair];
    const float scale = ldexpf(1.0f, 2 * g.level);
    const float inv = 1.0f / (255.0f * scale);
    // tree-edge bits (1 right, 2 down, 4 left, 8 up; 16 root), then in one
    // batch the slot words of both directions of every tree edge, the colours
    // of the pixel and its tree neighbours and the interval; then the run
    // prefixes
    const uint8_t a = adj[v];
    uint64_t wv[4], ww[4];
    float4 cw[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const bool e = (a >> d) & 1;
        const int64_t w = nbr(v, d, W);
        wv[d] = e ? rank_of.lw[4 * v + d] : 0;
        ww[d] = e ? rank_of.lw[4 * w + ((d + 2) & 3)] : 0;
        cw[d] = e ? img[w] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const float4 cv = img[v];
    // a pixel interval outside [0, dmax] or wider than max_width (counted by
    // the local phase in info, which makes the forest invalid) is clamped, so
    // that no later kernel reads a label outside the image row or writes past
    // the end of a volume row
    const int dm = g.dmax[pair];
    int l = plo ? plo[v] : 0;
    int h = plo ? phi[v] : dm;
    if (plo) {
        l = l < 0 ? 0 : (l > dm ? dm : l);
        h = h < l ? l : (h > dm ? dm : h);
        h = h - l + 1 > max_width ? l + max_width - 1 : h;
    }
    uint32_t rv[4], rw[4], kw[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const bool e = (a >> d) & 1;
        rv[d] = e ? (uint32_t)wv[d] + (uint32_t)rank_of.pr[wv[d] >> 32] : 0;
        rw[d] = e ? (uint32_t)ww[d] + (uint32_t)rank_of.pr[ww[d] >> 32] : 0;
        // key of the edge to every tree neighbour, taken from its lower pixel
        // id first as in the forest build (only the parent's is kept)
        kw[d] = d >= 2 ? edge_key(cw[d], cv, scale) : edge_key(cv, cw[d], scale);
    }
    // w is a child when the tour takes v -> w before w -> v (higher rank = earlier),
    // with (rank(v -> w) - rank(w -> v) + 1) / 2 nodes in its subtree; the
    // heavy child has the largest subtree (first in ascending pixel id on ties)
    const int order[4] = {3, 2, 0, 1};  // up, left, right, down: ascending pixel id
    int pd = -1, hd = -1;
    uint32_t bs = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int d = order[i];
        const bool e = (a >> d) & 1;
        if (e && rv[d] < rw[d]) pd = d;
        const uint32_t sz = e && rv[d] > rw[d] ? (rv[d] - rw[d] + 1) >> 1 : 0;
        if (sz > bs) {
            bs = sz;
            hd = d;
        }
    }
    int32_t par = -1;
    float wt = 0.f;
    uint64_t rvl = 0;
    if (!(a & kRootBit)) {
        uint32_t k = kw[0];
#pragma unroll
        for (int d = 1; d < 4; ++d) k = d == pd ? kw[d] : k;
        par = (int32_t)nbr(v, pd, W);
        wt = (float)k * inv;
    } else {
        const uint8_t t4 = a & 15;
        int32_t sz = 1;
        if (t4) {
            const int fd = first_dir(t4);
            uint32_t r0 = rv[0];
#pragma unroll
            for (int d = 1; d < 4; ++d) r0 = d == fd ? rv[d] : r0;
            sz = (int32_t)((r0 + 1) >> 1) + 1;
        }
        size[v] = sz;
        // low = tour length 2(sz-1), high = node count sz
        rvl = ((uint64_t)(uint32_t)sz << 32) | (uint32_t)(2 * (sz - 1));
    }
    parent[v] = par;
    wgt[v] = wt;
    rootval[v] = rvl;
    lo[v] = l;
    hi[v] = h;
    uint32_t code = (uint32_t)a | ((uint32_t)(l & 255) << 16) | ((uint32_t)(h & 255) << 24);
    if (pd >= 0) code |= (uint32_t)pd << 5;
    if (hd >= 0) code |= kHasHeavy | ((uint32_t)hd << 8);
    nrec[v] = make_uint2(code, __float_as_uint(wt));
    return rvl;
}

// One workgroup per scan tile of pixels, so the tile sums of the root data
// (the first half of the root-data scan) come out of the same launch.
constexpr int kParentThreads = kScanTile;
__global__ __launch_bounds__(kParentThreads) void k_parent(
    LevelGeom g, const float4 *__restrict__ img, Ranks rank_of, const uint8_t *__restrict__ adj,
    const int32_t *__restrict__ plo, const int32_t *__restrict__ phi, int max_width,
    int32_t *__restrict__ parent, int32_t *__restrict__ size, float *__restrict__ wgt,
    uint64_t *__restrict__ rootval, int32_t *__restrict__ lo, int32_t *__restrict__ hi,
    uint2 *__restrict__ nrec, uint64_t *__restrict__ tile_sum, int n_scan) {
    __shared__ uint64_t s_w[kParentThreads / 64];
    // each XCD takes a contiguous band of scan tiles (workgroups are dealt to
    // the XCDs in turn), so the rows above and below a tile were read through
    // the same L2
    const int per = (n_scan + kXcds - 1) / kXcds;
    const int tile = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    if (tile >= n_scan) return;
    const int64_t v = (int64_t)tile * kParentThreads + threadIdx.x;
    uint64_t x = 0;
    if (v < g.off[g.n_pairs])
        x = parent_of_pixel(v, g, img, rank_of, adj, plo, phi, max_width, parent, size, wgt,
                            rootval, lo, hi, nrec);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int i = 0; i < kParentThreads / 64; ++i) t += s_w[i];
        tile_sum[tile] = t;
    }
}

// --- 6. tour prefix sum: depth, light depth, preorder ---------------------------------
// Packed 64-bit tour value: bits 0-21 depth, 22-27 light depth, 28-63 down edges.
// The tour itself is stored as one byte per step (down or up, heavy or light
// edge) and widened to its packed value as the prefix sum reads it.
constexpr int kDepthBits = 22;
constexpr int kLdShift = 22;
constexpr int kDownShift = 28;
enum : uint8_t { kStepDownHeavy = 1, kStepDownLight = 2, kStepUpHeavy = 3, kStepUpLight = 4 };
struct TourStep {
    __device__ uint64_t operator()(uint8_t c) const {
        const uint64_t light = (c == kStepDownLight || c == kStepUpLight) ? 1 : 0;
        if (c == kStepDownHeavy || c == kStepDownLight)
            return (1ull << kDownShift) + (light << kLdShift) + 1ull;
        return c ? 0ull - (light << kLdShift) - 1ull : 0ull;
    }
};

__global__ void k_tour_scatter(LevelGeom g, const uint2 *__restrict__ nrec,
                               const int32_t *__restrict__ tree, const int32_t *__restrict__ size,
                               Ranks rank_of, const uint64_t *__restrict__ rootoff,
                               uint8_t *__restrict__ tourval, int32_t *__restrict__ posw,
                               int n_tiles, int32_t *__restrict__ info) {
    bool ok;
    int W;
    const int64_t v = tiled_pixel(g, n_tiles, &W, &ok);
    if (!ok) return;
    const uint32_t c = nrec[v].x;
    const uint8_t a = c & 15;
    if (!a) return;
    const int pd = code_pdir(c), hd = code_hdir(c);
    // loads in three batches: the pixel's own data and slot words, then the
    // root data, the parent's code and the run-end ranks, then the stores
    const int64_t root = tree[v];
    uint64_t wv[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) wv[d] = ((a >> d) & 1) ? rank_of.lw[4 * v + d] : 0;
    const uint32_t toff = (uint32_t)rootoff[root];
    const int64_t tlen = 2 * (int64_t)(size[root] - 1);
    const uint32_t cp = pd >= 0 ? nrec[nbr(v, pd, W)].x : 0;
    // v is its parent's heavy child when the parent's heavy direction points back at v
    const bool vheavy = pd >= 0 && code_hdir(cp) == ((pd + 2) & 3);
    uint32_t rk[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
        rk[d] = ((a >> d) & 1) ? (uint32_t)wv[d] + (uint32_t)rank_of.pr[wv[d] >> 32] : 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (!((a >> d) & 1)) continue;
        int64_t pos = (int64_t)toff + (tlen - 1 - (int64_t)rk[d]);
        const bool bad = pos < toff || pos >= (int64_t)toff + tlen;
        // the child of a down edge learns where its edge sits on the tour
        if (d != pd) posw[nbr(v, d, W)] = bad ? -1 : (int32_t)pos;
        if (bad) {
            info[HDP_INFO_ERROR] = 2;
            continue;
        }
        uint8_t step;
        if (d != pd)  // down edge v -> child
            step = d != hd ? kStepDownLight : kStepDownHeavy;
        else  // up edge v -> parent
            step = vheavy ? kStepUpHeavy : kStepUpLight;
        tourval[pos] = step;
    }
}

// Maximum over the active lanes of a wavefront, then one atomicMax.
__device__ __forceinline__ void wave_max_to(int32_t *dst, int32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        int32_t y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(dst, x);
}

__global__ void k_node_order(LevelGeom g, const uint2 *__restrict__ nrec,
                             const int32_t *__restrict__ tree, const int32_t *__restrict__ posw,
                             const uint64_t *__restrict__ rootoff,
                             const uint64_t *__restrict__ tourscan, int64_t tour_len,
                             int32_t *__restrict__ depth, int32_t *__restrict__ ld,
                             int32_t *__restrict__ seq, int n_tiles, int32_t *__restrict__ info) {
    bool inside;
    int Wt;
    const int64_t w = tiled_pixel(g, n_tiles, &Wt, &inside);
    int32_t dep = 0, l = 0;
    if (inside) {
        // two batches of loads: tree, node code and the tour position of the
        // edge parent -> w (left by the tour scatter); then the root data and
        // the tour prefix sum at that position
        const int64_t root = tree[w];
        const bool nonroot = code_pdir(nrec[w].x) >= 0;
        const int32_t pos = nonroot ? posw[w] : 0;
        const bool ok = !nonroot || (pos >= 0 && pos < tour_len);
        const uint64_t ro = rootoff[root];
        const uint64_t P = nonroot && ok ? tourscan[pos] : 0;
        const uint32_t toff = (uint32_t)ro, noff = (uint32_t)(ro >> 32);
        int32_t pre = (int32_t)noff;
        if (!ok) {
            info[HDP_INFO_ERROR] = 3;
            pre = 0;
        } else if (nonroot) {
            dep = (int32_t)(P & ((1ull << kDepthBits) - 1));
            l = (int32_t)((P >> kLdShift) & 63);
            const uint64_t down = P >> kDownShift;
            const uint32_t tidx = noff - (toff >> 1);  // trees before this one
            pre = (int32_t)(down + tidx);
        }
        depth[w] = dep;
        ld[w] = l;
        if (pre < 0 || pre >= g.off[g.n_pairs])
            info[HDP_INFO_ERROR] = 4;
        else
            seq[pre] = (int32_t)w;
    }
}

struct LdKey {
    const int32_t *ld;
    __device__ int operator()(int64_t, int32_t x) const { return ld[x] & 63; }
};

struct DigitKey {
    const int32_t *depth;
    int shift;
    __device__ int operator()(int64_t, int32_t x) const { return (depth[x] >> shift) & 255; }
};

// Rows: the stable partition of the preorder by light depth (counting
// scatter over the scanned per-tile histograms), and in block 0 the chain-phase
// table read from the same scanned histograms.
__global__ void k_phase_rows(const int32_t *__restrict__ seq, int64_t n, LdKey key,
                             const int32_t *__restrict__ offs, int64_t ntiles,
                             int32_t *__restrict__ node, int32_t *__restrict__ row,
                             int32_t *__restrict__ phase_ptr, int32_t *__restrict__ info) {
    const int k = threadIdx.x;
    const int64_t tile = band_tile(ntiles);
    if (tile < 0) return;
    if (tile == 0 && k <= HDP_MAX_PHASES) {
        int32_t v = offs[(int64_t)k * ntiles];  // rows with light depth < k
        phase_ptr[k] = v;
        // phases = 1 + largest light depth present: the first k with all rows below it
        int32_t prev = k > 0 ? offs[(int64_t)(k - 1) * ntiles] : 0;
        if (k > 0 && v == n && prev < n) info[HDP_INFO_N_PHASES] = k;
    }
    count_scatter_tile<64, 6>(seq, n, key, offs, ntiles, node, row, tile);
}

// Build statistics into info (one wavefront: lane r reads round r's flags).
__device__ __forceinline__ void finish_info(const int32_t *__restrict__ flags,
                                            const int32_t *__restrict__ ctr,
                                            int32_t *__restrict__ info, int width, int64_t n,
                                            const uint64_t *__restrict__ root_total) {
    const int r = threadIdx.x;
    const uint64_t bv = __ballot(r < 64 && flags[FLAG_BV + r] != 0);
    const uint64_t rk = __ballot(r < 64 && flags[FLAG_RANK + r] != 0);
    if (r != 0) return;
    info[HDP_INFO_LIVE_EDGES] = ctr[CTR_E];
    info[HDP_INFO_ACTIVE_COMPONENTS] = ctr[CTR_RALL];
    info[HDP_INFO_TOUR_RUNS] = ctr[CTR_RUNS];
    info[HDP_INFO_LIST_EDGES] = ctr[CTR_ET];
    // every tree of sz nodes has a tour of 2(sz - 1) slots
    info[HDP_INFO_N_TREES] = (int32_t)(n - (int64_t)((uint32_t)*root_total >> 1));
    info[HDP_INFO_MST_ROUNDS] = __popcll(bv);
    info[HDP_INFO_RANK_ROUNDS] = __popcll(rk);
    info[HDP_INFO_WIDTH] = width;
}

// --- 7. rows of the volume layout ---------------------------------------------------

// Per row r (coalesced writes) from its pixel v = node[r] (gathered reads:
// the node record, then the rows of the tree neighbours; consecutive rows
// are neighbouring pixels of a chain): parent row, heavy flag, edge weight,
// the rows of up to three light children in ascending pixel id, and the
// pixel's column and interval (read by the fused matching pass instead of the
// pixel arrays).  A heavy child is the row right after its parent's: the rows
// are the preorder split stably by light depth, and everything the preorder
// visits between a node and its heavy child lies below a light edge, while a
// light child cannot directly follow its parent (the parent's heavy child
// comes right after the parent in the parent's class).  Block 0 also writes
// the build statistics.
__global__ void k_rows(LevelGeom g, const int32_t *__restrict__ node,
                       const int32_t *__restrict__ row_of, const uint2 *__restrict__ nrec,
                       int32_t *__restrict__ prow, uint8_t *__restrict__ heavy,
                       int32_t *__restrict__ lc, float *__restrict__ rw, int32_t *__restrict__ rx,
                       int32_t *__restrict__ rlh, const int32_t *__restrict__ flags,
                       const int32_t *__restrict__ ctr, int32_t *__restrict__ info, int width,
                       const uint64_t *__restrict__ root_total) {
    // each XCD takes a contiguous band of row blocks (neighbouring chains of
    // the preorder, so their pixels' records come through the same L2)
    const int per = (int)(gridDim.x / kXcds);
    const int blk = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    const int64_t r = (int64_t)blk * kBlock + threadIdx.x;
    const int64_t n = g.off[g.n_pairs];
    if (blk == 0 && threadIdx.x < 64) finish_info(flags, ctr, info, width, n, root_total);
    if (r >= n) return;
    const int v = node[r];
    const uint2 rec = nrec[v];
    const uint32_t c = rec.x;
    const int pair = pair_of(g, v);
    const int W = g.W[pair];
    const int pd = code_pdir(c), hd = code_hdir(c);
    // rows of every tree neighbour (the parent among them), loaded together
    const int order[4] = {3, 2, 0, 1};  // up, left, right, down: ascending pixel id
    int rn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        rn[i] = ((c >> order[i]) & 1) ? row_of[nbr(v, order[i], W)] : -1;
    rw[r] = __uint_as_float(rec.y);
    rx[r] = (v - g.off[pair]) % W;
    rlh[r] = (int32_t)(((c >> 16) & 255) | (((c >> 24) & 255) << 16));
    int rp = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) rp = order[i] == pd ? rn[i] : rp;
    prow[r] = rp;
    heavy[r] = (rp >= 0 && rp == r - 1) ? 1 : 0;
    int k = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int d = order[i];
        if (!((c >> d) & 1) || d == pd || d == hd) continue;  // parent or heavy child
        if (k < 2) lc[(int64_t)k * n + r] = rn[i];
        ++k;
    }
    if (k > 2) info[HDP_INFO_ERROR] = 1;  // a root that is not its tree's smallest pixel
    for (; k < 2; ++k) lc[(int64_t)k * n + r] = -1;
}

// --- 8. canonical level order ------------------------------------------------------------

__global__ void k_iota(int32_t *__restrict__ a, int64_t n) {
    int64_t i = gtid();
    if (i < n) a[i] = (int32_t)i;
}

// level_ptr[k] = first position of depth k in the level order: every
// position where the depth steps up from d' to d writes the entries d'+1..d.
__global__ void k_level_ptr(const int32_t *__restrict__ order, const int32_t *__restrict__ depth,
                            int64_t n, int32_t *__restrict__ level_ptr,
                            int32_t *__restrict__ info) {
    int64_t i = gtid();
    if (i > n) return;
    int d = i < n ? depth[order[i]] : depth[order[n - 1]] + 1;
    int dp = i > 0 ? depth[order[i - 1]] : -1;
    for (int k = dp + 1; k <= d; ++k) level_ptr[k] = (int32_t)i;
    if (i == n) info[HDP_INFO_N_LEVELS] = d;
}


// --- learnable edge weights -----------------------------------------------------------------

__global__ void k_set_weights(int64_t n, const int32_t *__restrict__ node,
                              const int32_t *__restrict__ parent, const float *__restrict__ w,
                              float *__restrict__ wgt, float *__restrict__ rw) {
    int64_t r = gtid();
    if (r >= n) return;
    int v = node[r];
    float x = parent[v] >= 0 ? w[v] : 0.f;
    wgt[v] = x;
    rw[r] = x;
}

void launch_set_weights(const hdp_forest &f, const float *w, hipStream_t st) {
    k_set_weights<<<grid_for(f.n), kBlock, 0, st>>>(f.n, f.node, f.parent, w, f.wgt, f.rw);
}

// --- workspace -----------------------------------------------------------------------------

struct Bump {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (size_t)(count < 1 ? 1 : count);
        return p;
    }
};

struct TreeWs {
    int32_t *comp0, *lmin, *croot, *mnroot, *Rall, *At, *slot, *ctr, *flags;
    int32_t *size, *ld, *seq, *posw;
    uint64_t *cw, *best0, *best1, *E, *Et, *lw, *pr, *rootval, *tourval, *partial64, *root_total;
    uint8_t *tour8;
    uint32_t *C;
    uint2 *nrec;
    uint8_t *intree, *adj;
    int32_t *partial32, *hist, *sortA, *sortB;
    int32_t *hist2, *part2;  // counting sort of the 2n edge ids (literal forest)
};

static TreeWs carve_tree_ws(void *ws, int64_t n, size_t *bytes) {
    Bump b{reinterpret_cast<char *>(ws)};
    TreeWs t;
    int64_t ntiles = scan_tiles(n + 1) + 1;
    t.comp0 = b.take<int32_t>(n);
    t.lmin = b.take<int32_t>(n);
    t.croot = b.take<int32_t>(n);
    t.mnroot = b.take<int32_t>(n);
    t.Rall = b.take<int32_t>(n);
    t.At = b.take<int32_t>(2 * n);
    t.slot = b.take<int32_t>(2 * n);
    t.ctr = b.take<int32_t>(kCounters);
    t.flags = b.take<int32_t>(FLAG_WORDS);
    t.size = b.take<int32_t>(n);
    t.ld = b.take<int32_t>(n);
    t.seq = b.take<int32_t>(n);
    t.posw = b.take<int32_t>(n);
    t.cw = b.take<uint64_t>(n);
    t.best0 = b.take<uint64_t>(n);
    t.best1 = b.take<uint64_t>(n);
    t.E = b.take<uint64_t>(2 * n);
    t.Et = b.take<uint64_t>(2 * n);
    t.lw = b.take<uint64_t>(4 * n);
    t.pr = b.take<uint64_t>(2 * n);
    t.C = b.take<uint32_t>(2 * n);
    t.nrec = b.take<uint2>(n);
    t.rootval = b.take<uint64_t>(n);
    t.tourval = b.take<uint64_t>(2 * n);
    t.tour8 = b.take<uint8_t>(2 * n);
    t.partial64 = b.take<uint64_t>(scan_scratch(2 * n));
    t.root_total = b.take<uint64_t>(1);
    t.intree = b.take<uint8_t>(2 * n);
    t.adj = b.take<uint8_t>(n);
    t.partial32 = b.take<int32_t>(scan_scratch(256 * ntiles));
    t.hist = b.take<int32_t>(256 * ntiles);
    t.sortA = b.take<int32_t>(n);
    t.sortB = b.take<int32_t>(n);
    const int64_t etiles = scan_tiles(2 * n) + 1;
    t.hist2 = b.take<int32_t>(256 * etiles);
    t.part2 = b.take<int32_t>(scan_scratch(256 * etiles));
    *bytes = b.off + 256;
    return t;
}

size_t tree_workspace_bytes(int64_t n) {
    size_t bytes = 0;
    carve_tree_ws(nullptr, n, &bytes);
    return bytes;
}

static int ceil_log2(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}

template <int NB, int NBITS, typename KeyFn>
static void counting_sort(const int32_t *src, int32_t *dst, int32_t *pos_of, int64_t n, KeyFn key,
                          int32_t *hist, int32_t *partial32, hipStream_t st) {
    int64_t ntiles = scan_tiles(n);
    if (ntiles < 1) ntiles = 1;
    k_count_hist<NB><<<band_grid(ntiles), kBlock, 0, st>>>(src, n, key, hist, ntiles);
    device_scan<int32_t>(hist, hist, (int64_t)NB * ntiles, partial32, nullptr, false, st);
    k_count_scatter<NB, NBITS><<<band_grid(ntiles), kBlock, 0, st>>>(src, n, key, hist, ntiles, dst,
                                                                    pos_of);
}

void launch_build_tree(const float *img, const LevelGeom &g, const int32_t *plo,
                       const int32_t *phi, int max_width, int width, const int32_t *rank,
                       const hdp_forest &f, void *ws, hipStream_t st, bool literal, int beta_num,
                       int beta_den) {
    int64_t n = g.off[g.n_pairs];
    size_t bytes;
    TreeWs t = carve_tree_ws(ws, n, &bytes);
    const float4 *im = reinterpret_cast<const float4 *>(img);
    unsigned gn = grid_for(n);

    // Round bounds.  After the tile-local phase every component that still has
    // an edge owns a tile-border pixel, and the number of such components at
    // least halves per global round.  A tour's contracted list has at most one
    // entry per directed tree edge that crosses a tile border, plus its end.
    int64_t border_px = 0, max_list = 2, runs_bound = 0;
    unsigned n_tiles = (unsigned)g.toff[g.n_pairs];
    for (int p = 0; p < g.n_pairs; ++p) {
        int H = g.H[p], W = g.W[p];
        int tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
        for (int j = 0; j < ty; ++j)
            for (int i = 0; i < tx; ++i) {
                int64_t tw = W - i * kTile < kTile ? W - i * kTile : kTile;
                int64_t th = H - j * kTile < kTile ? H - j * kTile : kTile;
                int64_t inner = (tw > 2 ? tw - 2 : 0) * (th > 2 ? th - 2 : 0);
                border_px += tw * th - inner;
            }
        int64_t crossing = (int64_t)H * (tx - 1) + (int64_t)W * (ty - 1);
        if (2 * crossing + 2 > max_list) max_list = 2 * crossing + 2;
        runs_bound += 2 * crossing + 1;
    }
    unsigned g_edges = grid_for(2 * n) < (unsigned)kGridCap ? grid_for(2 * n) : kGridCap;
    unsigned g_roots = grid_for(border_px) < (unsigned)kGridCap ? grid_for(border_px) : kGridCap;

    // intervals and bound the layout kernels see: the pixel intervals (in the
    // regime every tree keeps its pixels' interval), or the trees' intervals
    const int32_t *plo_f = plo, *phi_f = phi;
    int mw_f = max_width;
    k_tree_init<<<1, FLAG_WORDS, 0, st>>>(t.flags, t.ctr, f.info);
    if (literal) {
        // 1-3 (literal forest): keys and filter, stable sort of the edge ids by
        // key (8 bits a pass; ids ascending among equal keys), the sequential
        // process, then each pixel's tree, smallest pixel and tree interval
        uint32_t *ekey = reinterpret_cast<uint32_t *>(t.cw);
        int32_t *uf = t.Rall, *usz = t.slot;
        int32_t *tlo = reinterpret_cast<int32_t *>(t.best0), *thi = tlo + n;
        int32_t *plo2 = reinterpret_cast<int32_t *>(t.best1), *phi2 = plo2 + n;
        // keys below 2^16 (colour keys to layer 4), 2^24, or 31-bit ranks
        const int passes = rank ? 4 : (255ll << (2 * g.level)) < 0xFFFF ? 2 : 3;
        const uint32_t sentinel = passes == 4 ? 0xFFFFFFFFu : (1u << (8 * passes)) - 1u;
        k_seq_edges<<<gn, kBlock, 0, st>>>(im, g, plo, phi, rank, sentinel, ekey, uf, usz, tlo,
                                           thi, t.croot, t.lmin, t.intree, f.info);
        int32_t *src = reinterpret_cast<int32_t *>(t.E), *dst = src + 2 * n;
        k_iota<<<grid_for(2 * n), kBlock, 0, st>>>(src, 2 * n);
        for (int pass = 0; pass < passes; ++pass) {
            counting_sort<256, 8>(src, dst, nullptr, 2 * n, EdgeDigit{ekey, 8 * pass}, t.hist2,
                                  t.part2, st);
            int32_t *tmp = src;
            src = dst;
            dst = tmp;
        }
        k_seq_kruskal<<<1, kSeqThreads, 0, st>>>(src, ekey, 2 * n, sentinel, g, beta_num,
                                                  beta_den, uf, usz, tlo, thi, t.intree);
        k_seq_roots<<<gn, kBlock, 0, st>>>(uf, tlo, thi, n, width, t.comp0, t.lmin, plo2, phi2,
                                           f.info);
        plo_f = plo2;
        phi_f = phi2;
        mw_f = width;
    } else {
        // 1-2: spanning forest (tile-local phase, full-grid rounds, one-workgroup tail)
        k_local_msf<<<n_tiles, kLocalThreads, 0, st>>>(im, g, plo, phi, max_width, rank, t.comp0, t.cw,
                                                       t.best0, t.best1, t.lmin, t.croot, t.mnroot,
                                                       t.intree, t.E, t.Rall, t.ctr, f.info);
        int bv_rounds = ceil_log2(border_px) + 1;
        if (bv_rounds > kBvGridRounds) bv_rounds = kBvGridRounds;
        if (bv_rounds < 1) bv_rounds = 1;
        // A layer without intervals (one spanning tree per pair) with few tile-border
        // pixels leaves a contracted graph that the one-workgroup tail takes whole
        // (about 1.5 live edges per border pixel; in LDS when it fits, else in the
        // tail's global-memory mode): no full-grid rounds are launched.
        if (!plo && border_px <= kTopAloneBorderPx) bv_rounds = 0;
        for (int r = 0; r < bv_rounds; ++r) {
            uint64_t *bc = (r & 1) ? t.best1 : t.best0, *bn = (r & 1) ? t.best0 : t.best1;
            if (r > 0)  // round 0's minimum edges come from the tile-local phase
                k_gbv_minedge<false><<<g_edges, kBlock, 0, st>>>(r, t.flags, t.ctr, g, t.E, t.comp0, t.cw,
                                                          bc, f.info);
            k_gbv_hook<<<g_roots, kBlock, 0, st>>>(r, t.flags, t.ctr, g, t.Rall, t.comp0, t.cw, bc, bn,
                                                   t.intree, f.info);
        }
        if (bv_rounds > 0)  // without rounds every listed edge is live: the tail reads the list
            k_gbv_compact<<<g_edges, kBlock, 0, st>>>(bv_rounds, t.flags, t.ctr, g, t.E, t.comp0, t.cw,
                                                  t.Et, f.info);
        // Rounds on the compacted list (each skipped once a round hooked nothing),
        // launched where the tail would otherwise take more live edges than its
        // LDS holds: after the full-grid rounds about one live edge per 6 border
        // pixels is left on a layer without intervals, one per 64 with intervals
        // (measured).  Elsewhere their launches would cost more than they save.
        const int64_t est_left = plo ? border_px / 64 : border_px / 6;
        const int list_rounds = bv_rounds > 0 && est_left > kTE / 2 ? kBvListRounds : 0;
        const unsigned g_list = g_edges < 512u ? g_edges : 512u;
        for (int r = bv_rounds; r < bv_rounds + list_rounds; ++r) {
            uint64_t *bc = (r & 1) ? t.best1 : t.best0, *bn = (r & 1) ? t.best0 : t.best1;
            k_gbv_minedge<true><<<g_list, kBlock, 0, st>>>(r, t.flags, t.ctr, g, t.Et, t.comp0, t.cw,
                                                           bc, f.info);
            k_gbv_lhook<<<g_list, kBlock, 0, st>>>(r, t.flags, t.ctr, g, t.Et, t.comp0, t.cw, bc, bn,
                                                   t.intree, f.info);
        }
        k_gbv_tail<<<1, kLocalThreads, 0, st>>>(bv_rounds + list_rounds, t.flags, t.ctr, g, t.E, t.Et,
                                                t.comp0, t.cw, t.Rall, t.croot, t.best0, t.best1,
                                                t.intree, f.info);
        // 3: roots
        k_gbv_final<<<g_roots, kBlock, 0, st>>>(t.ctr, t.Rall, t.cw, t.lmin, t.croot, t.mnroot, f.info);
    }
    k_set_tree<<<gn, kBlock, 0, st>>>(t.comp0, t.croot, t.lmin, t.mnroot, t.intree, g, f.tree,
                                      t.adj, f.info);
    // 4: Euler tour ranks
    k_tour_local<<<n_tiles, kTourThreads, 0, st>>>(g, t.adj, t.lw, t.C, t.ctr, f.info);
    k_tour_link<<<g_edges, kBlock, 0, st>>>(t.ctr, t.C, t.lw, t.pr);
    int rk_rounds = ceil_log2(max_list) + 1;
    if (rk_rounds < 1) rk_rounds = 1;
    // With intervals (in the regime) the trees are small (the longest
    // contracted list of the 1344x1104 pair's level 0 has under a thousand
    // entries): one launch, and the tail finishes any longer list.
    if (plo && !literal && rk_rounds > kRankJumps) rk_rounds = kRankJumps;
    // Without intervals every pair's forest is one spanning tree (one tour), so
    // the contracted list is bounded by runs_bound: a list that fits the LDS
    // tail needs no full-grid rounds at all.
    if (!plo && runs_bound <= kTA) rk_rounds = 0;
    rk_rounds = (rk_rounds + kRankJumps - 1) / kRankJumps;  // launches of kRankJumps jumps
    for (int r = 0; r < rk_rounds; ++r)
        k_rank_round<<<g_edges, kBlock, 0, st>>>(r, t.flags, t.ctr, t.pr);
    if (rk_rounds > 0)  // without rounds the tail reads the whole list itself
        k_rank_compact<<<g_edges, kBlock, 0, st>>>(rk_rounds, t.flags, t.ctr, t.pr, t.At);
    k_rank_tail<<<1, kLocalThreads, 0, st>>>(rk_rounds, t.flags, t.ctr, t.At, t.slot, t.pr,
                                             f.info);
    Ranks rk{t.lw, t.pr};
    // 5: parents, subtree sizes, heavy children
    const unsigned n_scan = (unsigned)(scan_tiles(n) < 1 ? 1 : scan_tiles(n));
    k_parent<<<kXcds * ((n_scan + kXcds - 1) / kXcds), kParentThreads, 0, st>>>(
        g, im, rk, t.adj, plo_f, phi_f, mw_f, f.parent, t.size, f.wgt, t.rootval, f.lo, f.hi,
        t.nrec,
        t.partial64, (int)n_scan);
    // 6: tour offsets (the root-data scan, tile sums from k_parent), tour
    // values, prefix sum, per-node depth / light depth / preorder
    scan_sums_and_apply(t.rootval, t.rootval, n, t.partial64, (int64_t)n_scan, t.root_total,
                        false, st, WidenSame());
    k_tour_scatter<<<tiled_grid((int)n_tiles), kBlock, 0, st>>>(
        g, t.nrec, f.tree, t.size, rk, t.rootval, t.tour8, t.posw, (int)n_tiles, f.info);
    int64_t tour_len = 2 * n;  // upper bound; entries past the real length are never read
    device_scan<uint64_t>(t.tour8, t.tourval, tour_len, t.partial64, nullptr, true, st, TourStep());
    k_node_order<<<tiled_grid((int)n_tiles), kBlock, 0, st>>>(
        g, t.nrec, f.tree, t.posw, t.rootval, t.tourval, tour_len, f.depth, t.ld, t.seq,
        (int)n_tiles, f.info);
    // 7: rows (stable partition of the preorder by light depth)
    {
        int64_t ntiles = scan_tiles(n);
        if (ntiles < 1) ntiles = 1;
        LdKey key{t.ld};
        k_count_hist<64><<<band_grid(ntiles), kBlock, 0, st>>>(t.seq, n, key, t.hist, ntiles);
        device_scan<int32_t>(t.hist, t.hist, 64 * ntiles, t.partial32, nullptr, false, st);
        k_phase_rows<<<band_grid(ntiles), kBlock, 0, st>>>(t.seq, n, key, t.hist, ntiles, f.node,
                                                          f.row, f.phase_ptr, f.info);
    }
    k_rows<<<kXcds * ((gn + kXcds - 1) / kXcds), kBlock, 0, st>>>(
        g, f.node, f.row, t.nrec, f.prow, f.heavy, f.lc, f.rw, f.rx, f.rlh, t.flags, t.ctr, f.info,
        width, t.root_total);
}

// 8: level order (stable LSD radix sort of ids by depth) and level_ptr
void launch_level_order(const hdp_forest &f, void *ws, hipStream_t st) {
    int64_t n = f.n;
    size_t bytes;
    TreeWs t = carve_tree_ws(ws, n, &bytes);
    k_iota<<<grid_for(n), kBlock, 0, st>>>(t.sortA, n);
    int32_t *src = t.sortA, *dst = t.sortB;
    int passes = ceil_log2(n) <= 8 ? 1 : ceil_log2(n) <= 16 ? 2 : 3;
    for (int pass = 0; pass < passes; ++pass) {
        int32_t *out = pass == passes - 1 ? f.order : dst;
        counting_sort<256, 8>(src, out, nullptr, n, DigitKey{f.depth, 8 * pass}, t.hist,
                              t.partial32, st);
        src = out;
        dst = (out == t.sortB) ? t.sortA : t.sortB;
    }
    k_level_ptr<<<grid_for(n + 1), kBlock, 0, st>>>(f.order, f.depth, n, f.level_ptr, f.info);
}

}  // namespace hdp
