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

// --- 1. edge keys ------------------------------------------------------------

__global__ void k_edge_keys(const float4 *__restrict__ img, LevelGeom g,
                            const int32_t *__restrict__ plo, const int32_t *__restrict__ phi,
                            int max_width, uint32_t *__restrict__ key, int32_t *__restrict__ info) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    PixelPos p = pixel_pos(g, (int)v);
    float scale = ldexpf(1.0f, 2 * g.level);
    float4 a = img[v];
    if (plo) {
        int lo = plo[v], hi = phi[v];
        if (lo < 0 || hi < lo || hi > g.dmax[p.pair] || hi - lo + 1 > max_width)
            atomicAdd(&info[HDP_INFO_BAD_INTERVAL], 1);
    }
    for (int dir = 0; dir < 2; ++dir) {
        bool inside = dir == 0 ? p.x + 1 < p.W : p.y + 1 < p.H;
        uint32_t k = kNoKey;
        if (inside) {
            int64_t q = dir == 0 ? v + 1 : v + p.W;
            if (!plo || (plo[v] == plo[q] && phi[v] == phi[q])) {
                float4 b = img[q];
                float m = fmaxf(fmaxf(fabsf(a.x - b.x), fabsf(a.y - b.y)), fabsf(a.z - b.z));
                k = __float2uint_rn(m * scale);
            }
        }
        key[2 * v + dir] = k;
    }
}

// --- 2. Boruvka ----------------------------------------------------------------

__global__ void k_bv_init(int32_t *__restrict__ comp, int32_t *__restrict__ nxt,
                          uint64_t *__restrict__ best, int32_t *__restrict__ mn,
                          uint8_t *__restrict__ intree, int64_t n, int32_t *__restrict__ flags,
                          int32_t *__restrict__ info) {
    int64_t v = gtid();
    if (v < FLAG_WORDS) flags[v] = 0;
    if (v < HDP_INFO_WORDS && v != HDP_INFO_BAD_INTERVAL) info[v] = 0;
    if (v >= n) return;
    comp[v] = (int32_t)v;
    nxt[v] = (int32_t)v;
    best[v] = kNoEdge;
    mn[v] = 0x7fffffff;
    intree[2 * v] = 0;
    intree[2 * v + 1] = 0;
}

__global__ void k_info_clear(int32_t *__restrict__ info) {
    if (threadIdx.x == 0) info[HDP_INFO_BAD_INTERVAL] = 0;
}

__global__ void k_bv_minedge(int round, const int32_t *__restrict__ flags, LevelGeom g,
                             uint32_t *__restrict__ key, const int32_t *__restrict__ comp,
                             uint64_t *__restrict__ best) {
    if (round > 0 && flags[FLAG_BV + round - 1] == 0) return;
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    uint2 kk = reinterpret_cast<const uint2 *>(key)[v];
    if (kk.x == kNoKey && kk.y == kNoKey) return;
    int cu = comp[v];
    for (int dir = 0; dir < 2; ++dir) {
        uint32_t k = dir == 0 ? kk.x : kk.y;
        if (k == kNoKey) continue;
        int64_t q = dir == 0 ? v + 1 : v + g.W[pair_of(g, (int)v)];
        int cq = comp[q];
        if (cq == cu) {  // both ends already in one component: never needed again
            key[2 * v + dir] = kNoKey;
            continue;
        }
        uint64_t k64 = ((uint64_t)k << 32) | (uint64_t)(2 * v + dir);
        if (best[cu] > k64) atomicMin((unsigned long long *)&best[cu], (unsigned long long)k64);
        if (best[cq] > k64) atomicMin((unsigned long long *)&best[cq], (unsigned long long)k64);
    }
}

__global__ void k_bv_hook(int round, int32_t *__restrict__ flags, LevelGeom g,
                          const uint64_t *__restrict__ best, const int32_t *__restrict__ comp,
                          int32_t *__restrict__ nxt, uint8_t *__restrict__ intree) {
    if (round > 0 && flags[FLAG_BV + round - 1] == 0) return;
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    if (comp[v] != v) return;
    uint64_t b = best[v];
    if (b == kNoEdge) return;
    uint32_t e = (uint32_t)b;
    int p = (int)(e >> 1);
    int q = (e & 1) ? p + g.W[pair_of(g, p)] : p + 1;
    int cp = comp[p], cq = comp[q];
    int other = cp == v ? cq : cp;
    intree[e] = 1;
    if (best[other] == b && v < other) return;  // mutual choice: the smaller id stays root
    nxt[v] = other;
    flags[FLAG_BV + round] = 1;
}

__global__ void k_bv_compress(int round, const int32_t *__restrict__ flags,
                              int32_t *__restrict__ comp, int32_t *__restrict__ nxt,
                              uint64_t *__restrict__ best, int64_t n, int32_t *__restrict__ info) {
    if (flags[FLAG_BV + round] == 0) return;
    int64_t v = gtid();
    if (v >= n) return;
    int c = comp[v];
    int r = c;
    int s = nxt[r];
    // the hook pointers form a forest, so the walk ends at a root; the bound
    // only guards against a broken invariant
    for (int64_t it = 0; s != r && it < n; ++it) {
        r = s;
        s = nxt[r];
    }
    if (s != r) info[HDP_INFO_ERROR] = 1;
    if (c != r) nxt[c] = r;  // path shortcut (any value written is an ancestor)
    comp[v] = r;
    best[v] = kNoEdge;
}

// --- 3. roots -------------------------------------------------------------------

// Smallest pixel id of every component.  Lanes of a wavefront that share a
// component (the common case: components are large and pixels contiguous)
// combine first, so one atomic per wavefront and component reaches memory.
__global__ void k_rootmin(const int32_t *__restrict__ comp, int32_t *__restrict__ mn, int64_t n) {
    __shared__ int s_c0, s_diff;
    int64_t v = gtid();
    bool valid = v < n;
    int c = valid ? comp[v] : -1;
    if (threadIdx.x == 0) { s_c0 = c; s_diff = 0; }
    __syncthreads();
    if (valid && c != s_c0) s_diff = 1;
    __syncthreads();
    if (!s_diff) {
        // the whole workgroup lies in one component; thread 0 holds the smallest id
        if (threadIdx.x == 0 && valid && mn[c] > (int32_t)v) atomicMin(&mn[c], (int32_t)v);
        return;
    }
    int c0 = __shfl(c, 0, 64);
    uint64_t same = __ballot(c == c0);
    uint64_t act = __ballot(valid);
    if (same == act) {
        if ((threadIdx.x & 63) == 0 && valid && mn[c0] > (int32_t)v) atomicMin(&mn[c0], (int32_t)v);
        return;
    }
    if (valid && mn[c] > (int32_t)v) atomicMin(&mn[c], (int32_t)v);
}

__global__ void k_set_tree(const int32_t *__restrict__ comp, const int32_t *__restrict__ mn,
                           const uint8_t *__restrict__ intree, LevelGeom g,
                           int32_t *__restrict__ tree, uint8_t *__restrict__ adj,
                           int32_t *__restrict__ info) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    int t = mn[comp[v]];
    tree[v] = t;
    if (t == v) atomicAdd(&info[HDP_INFO_N_TREES], 1);
    PixelPos p = pixel_pos(g, (int)v);
    uint8_t a = 0;
    if (intree[2 * v]) a |= 1;
    if (intree[2 * v + 1]) a |= 2;
    if (p.x > 0 && intree[2 * (v - 1)]) a |= 4;
    if (p.y > 0 && intree[2 * (v - p.W) + 1]) a |= 8;
    adj[v] = a;
}

// --- 4. Euler tour ranking ------------------------------------------------------

__device__ __forceinline__ int64_t nbr(int64_t v, int d, int W) {
    return d == 0 ? v + 1 : d == 1 ? v + W : d == 2 ? v - 1 : v - W;
}

__device__ __forceinline__ int first_dir(uint8_t a) { return __ffs((int)a) - 1; }

// slot 4v+d = directed tree edge from v in direction d.  Packed word:
// high 32 bits = next slot (-1 end of tour, -2 not an edge), low 32 = distance.
__global__ void k_euler_init(LevelGeom g, const uint8_t *__restrict__ adj,
                             const int32_t *__restrict__ tree, uint64_t *__restrict__ pr) {
    int64_t s = gtid();
    int64_t n = g.off[g.n_pairs];
    if (s >= 4 * n) return;
    int64_t v = s >> 2;
    int d = (int)(s & 3);
    uint8_t av = adj[v];
    if (!((av >> d) & 1)) {
        pr[s] = ((uint64_t)0xFFFFFFFEu << 32);
        return;
    }
    int W = g.W[pair_of(g, (int)v)];
    int64_t w = nbr(v, d, W);
    uint8_t aw = adj[w];
    int rd = d ^ 2, d2 = rd;
    for (int k = 1; k <= 4; ++k) {
        d2 = (rd + k) & 3;
        if ((aw >> d2) & 1) break;
    }
    int64_t succ = 4 * w + d2;
    bool end = tree[w] == w && d2 == first_dir(aw);
    if (end)
        pr[s] = ((uint64_t)0xFFFFFFFFu << 32);
    else
        pr[s] = ((uint64_t)(uint32_t)succ << 32) | 1u;
}

__global__ void k_rank_round(int round, int32_t *__restrict__ flags, uint64_t *__restrict__ pr,
                             int64_t n4) {
    if (round > 0 && flags[FLAG_RANK + round - 1] == 0) return;
    int64_t s = gtid();
    if (s >= n4) return;
    uint64_t P = __hip_atomic_load(&pr[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t nx = (int32_t)(P >> 32);
    if (nx < 0) return;
    uint64_t Q = __hip_atomic_load(&pr[nx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t nn = (int32_t)(Q >> 32);
    uint32_t dist = (uint32_t)P + (uint32_t)Q;
    __hip_atomic_store(&pr[s], ((uint64_t)(uint32_t)nn << 32) | dist, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if (nn >= 0) flags[FLAG_RANK + round] = 1;
}

__device__ __forceinline__ uint32_t rank_of(const uint64_t *pr, int64_t s) {
    return (uint32_t)pr[s];
}

// parent, subtree size and edge weight of the child side of every tree edge.
// (edge weights are recomputed from the image: the key array no longer holds
// the keys of edges that became internal during the spanning-forest rounds)
__global__ void k_parent(LevelGeom g, const uint8_t *__restrict__ intree,
                         const float4 *__restrict__ img, const uint64_t *__restrict__ pr,
                         int32_t *__restrict__ parent, int32_t *__restrict__ size,
                         float *__restrict__ wgt) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    int W = g.W[pair_of(g, (int)v)];
    float inv = 1.0f / (255.0f * ldexpf(1.0f, 2 * g.level));
    for (int dir = 0; dir < 2; ++dir) {
        int64_t e = 2 * v + dir;
        if (!intree[e]) continue;
        int64_t w = dir == 0 ? v + 1 : v + W;
        uint32_t rv = rank_of(pr, 4 * v + dir);
        uint32_t rw = rank_of(pr, 4 * w + (dir + 2));
        int64_t child, par;
        uint32_t sz;
        if (rv > rw) { child = w; par = v; sz = (rv - rw + 1) >> 1; }
        else { child = v; par = w; sz = (rw - rv + 1) >> 1; }
        float4 a = img[v], b = img[w];
        float m = fmaxf(fmaxf(fabsf(a.x - b.x), fabsf(a.y - b.y)), fabsf(a.z - b.z));
        float k = (float)__float2uint_rn(m * ldexpf(1.0f, 2 * g.level));
        parent[child] = (int32_t)par;
        size[child] = (int32_t)sz;
        wgt[child] = k * inv;
    }
}

__global__ void k_root_info(int64_t n, const int32_t *__restrict__ tree,
                            const uint8_t *__restrict__ adj, const uint64_t *__restrict__ pr,
                            int32_t *__restrict__ parent, int32_t *__restrict__ size,
                            float *__restrict__ wgt, uint64_t *__restrict__ rootval) {
    int64_t v = gtid();
    if (v >= n) return;
    uint64_t rv = 0;
    if (tree[v] == v) {
        parent[v] = -1;
        wgt[v] = 0.f;
        uint8_t a = adj[v];
        int32_t sz = a ? (int32_t)((rank_of(pr, 4 * v + first_dir(a)) + 1) >> 1) + 1 : 1;
        size[v] = sz;
        // packed for one scan: low = tour length 2(sz-1), high = node count sz
        rv = ((uint64_t)(uint32_t)sz << 32) | (uint32_t)(2 * (sz - 1));
    }
    rootval[v] = rv;
}

// --- 5. heavy child ----------------------------------------------------------------

__global__ void k_heavy(LevelGeom g, const uint8_t *__restrict__ adj,
                        const int32_t *__restrict__ parent, const int32_t *__restrict__ size,
                        int32_t *__restrict__ heavy_child) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    int W = g.W[pair_of(g, (int)v)];
    uint8_t a = adj[v];
    const int order[4] = {3, 2, 0, 1};  // up, left, right, down: ascending pixel id
    int best = -1, bs = -1;
    for (int i = 0; i < 4; ++i) {
        int d = order[i];
        if (!((a >> d) & 1)) continue;
        int64_t w = nbr(v, d, W);
        if (parent[w] != v) continue;
        if (size[w] > bs) { bs = size[w]; best = (int)w; }
    }
    heavy_child[v] = best;
}

// --- 6. tour prefix sum: depth, light depth, preorder ---------------------------------
// Packed 64-bit tour value: bits 0-21 depth, 22-27 light depth, 28-63 down edges.
constexpr int kDepthBits = 22;
constexpr int kLdShift = 22;
constexpr int kDownShift = 28;

__global__ void k_tour_scatter(LevelGeom g, const uint8_t *__restrict__ adj,
                               const int32_t *__restrict__ tree, const int32_t *__restrict__ parent,
                               const int32_t *__restrict__ size,
                               const int32_t *__restrict__ heavy_child,
                               const uint64_t *__restrict__ pr, const uint64_t *__restrict__ rootoff,
                               uint64_t *__restrict__ tourval, int32_t *__restrict__ info) {
    int64_t s = gtid();
    int64_t n = g.off[g.n_pairs];
    if (s >= 4 * n) return;
    int64_t v = s >> 2;
    int d = (int)(s & 3);
    if (!((adj[v] >> d) & 1)) return;
    int W = g.W[pair_of(g, (int)v)];
    int64_t w = nbr(v, d, W);
    int64_t root = tree[v];
    uint32_t toff = (uint32_t)rootoff[root];
    int64_t tlen = 2 * (int64_t)(size[root] - 1);
    int64_t pos = (int64_t)toff + (tlen - 1 - (int64_t)rank_of(pr, s));
    if (pos < toff || pos >= (int64_t)toff + tlen) {
        info[HDP_INFO_ERROR] = 2;
        return;
    }
    uint64_t val;
    if (parent[w] == v) {  // down edge v -> w
        uint64_t light = heavy_child[v] != w ? 1 : 0;
        val = (1ull << kDownShift) + (light << kLdShift) + 1ull;
    } else {  // up edge v -> parent w
        uint64_t light = heavy_child[w] != v ? 1 : 0;
        val = 0ull - (light << kLdShift) - 1ull;
    }
    tourval[pos] = val;
}

// Maximum over the active lanes of a wavefront, then one atomicMax.
__device__ __forceinline__ void wave_max_to(int32_t *dst, int32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        int32_t y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(dst, x);
}

__global__ void k_node_order(LevelGeom g, const uint8_t *__restrict__ adj,
                             const int32_t *__restrict__ tree, const int32_t *__restrict__ parent,
                             const uint64_t *__restrict__ pr, const uint64_t *__restrict__ rootoff,
                             const int32_t *__restrict__ size, const uint64_t *__restrict__ tourscan,
                             int32_t *__restrict__ depth, int32_t *__restrict__ ld,
                             int32_t *__restrict__ gpre, int32_t *__restrict__ info) {
    int64_t w = gtid();
    int32_t dep = 0, l = 0;
    if (w < g.off[g.n_pairs]) {
        int64_t root = tree[w];
        uint64_t ro = rootoff[root];
        uint32_t toff = (uint32_t)ro, noff = (uint32_t)(ro >> 32);
        int32_t pre = (int32_t)noff;
        if (root != w) {
            int64_t p = parent[w];
            int W = g.W[pair_of(g, (int)w)];
            // direction of the edge p -> w (a one-pixel-wide image has vertical edges only)
            int d = W == 1 ? (w > p ? 1 : 3) : w == p + 1 ? 0 : w == p + W ? 1 : w == p - 1 ? 2 : 3;
            int64_t tlen = 2 * (int64_t)(size[root] - 1);
            int64_t pos = (int64_t)toff + (tlen - 1 - (int64_t)rank_of(pr, 4 * p + d));
            if (pos < toff || pos >= (int64_t)toff + tlen) {
                info[HDP_INFO_ERROR] = 3;
                pre = 0;
            } else {
                uint64_t P = tourscan[pos];
                dep = (int32_t)(P & ((1ull << kDepthBits) - 1));
                l = (int32_t)((P >> kLdShift) & 63);
                uint64_t down = P >> kDownShift;
                uint32_t tidx = noff - (toff >> 1);  // trees before this one
                pre = (int32_t)(down + tidx);
            }
        }
        depth[w] = dep;
        ld[w] = l;
        gpre[w] = pre;
    }
}

__global__ void k_scatter_seq(const int32_t *__restrict__ gpre, int32_t *__restrict__ seq,
                              int64_t n, int32_t *__restrict__ info) {
    int64_t v = gtid();
    if (v >= n) return;
    int32_t q = gpre[v];
    if (q < 0 || q >= n) {
        info[HDP_INFO_ERROR] = 4;
        return;
    }
    seq[q] = (int32_t)v;
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

__global__ void k_phase_ptr(const int32_t *__restrict__ offs, int64_t ntiles, int64_t n,
                            int32_t *__restrict__ phase_ptr, int32_t *__restrict__ info) {
    int k = threadIdx.x;
    if (k > HDP_MAX_PHASES) return;
    int32_t v = offs[(int64_t)k * ntiles];  // rows with light depth < k
    phase_ptr[k] = v;
    // phases = 1 + largest light depth present: the first k with all rows below it
    int32_t prev = k > 0 ? offs[(int64_t)(k - 1) * ntiles] : 0;
    if (k > 0 && v == n && prev < n) info[HDP_INFO_N_PHASES] = k;
}

// --- 7. rows of the volume layout ---------------------------------------------------

__global__ void k_rows(LevelGeom g, const int32_t *__restrict__ node,
                       const int32_t *__restrict__ row_of, const int32_t *__restrict__ parent,
                       const float *__restrict__ wgt, const int32_t *__restrict__ heavy_child,
                       const uint8_t *__restrict__ adj, int32_t *__restrict__ prow,
                       uint8_t *__restrict__ heavy, int32_t *__restrict__ lc,
                       float *__restrict__ rw) {
    int64_t r = gtid();
    int64_t n = g.off[g.n_pairs];
    if (r >= n) return;
    int64_t v = node[r];
    int64_t p = parent[v];
    prow[r] = p >= 0 ? row_of[p] : -1;
    heavy[r] = (p >= 0 && heavy_child[p] == v) ? 1 : 0;
    rw[r] = wgt[v];
    int W = g.W[pair_of(g, (int)v)];
    uint8_t a = adj[v];
    const int order[4] = {3, 2, 0, 1};
    int k = 0;
    int hc = heavy_child[v];
    for (int i = 0; i < 4; ++i) {
        int d = order[i];
        if (!((a >> d) & 1)) continue;
        int64_t w = nbr(v, d, W);
        if (parent[w] != v || w == hc) continue;
        if (k < 3) lc[(int64_t)k * n + r] = row_of[w];
        ++k;
    }
    for (; k < 3; ++k) lc[(int64_t)k * n + r] = -1;
}

__global__ void k_intervals(LevelGeom g, const int32_t *__restrict__ plo,
                            const int32_t *__restrict__ phi, int32_t *__restrict__ lo,
                            int32_t *__restrict__ hi) {
    int64_t v = gtid();
    if (v >= g.off[g.n_pairs]) return;
    if (plo) {
        lo[v] = plo[v];
        hi[v] = phi[v];
    } else {
        lo[v] = 0;
        hi[v] = g.dmax[pair_of(g, (int)v)];
    }
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

__global__ void k_finish_info(const int32_t *__restrict__ flags, int32_t *__restrict__ info,
                              int width) {
    if (threadIdx.x != 0) return;
    int bv = 0, rk = 0;
    for (int r = 0; r < 64; ++r) {
        bv += flags[FLAG_BV + r] ? 1 : 0;
        rk += flags[FLAG_RANK + r] ? 1 : 0;
    }
    info[HDP_INFO_MST_ROUNDS] = bv;
    info[HDP_INFO_RANK_ROUNDS] = rk;
    info[HDP_INFO_WIDTH] = width;
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
    uint32_t *key;
    int32_t *comp, *nxt, *mn, *flags, *size, *heavy_child, *ld, *gpre, *seq;
    uint64_t *best, *pr, *rootval, *tourval, *partial64;
    uint8_t *intree, *adj;
    int32_t *partial32, *hist, *sortA, *sortB, *cnt;
};

static TreeWs carve_tree_ws(void *ws, int64_t n, size_t *bytes) {
    Bump b{reinterpret_cast<char *>(ws)};
    TreeWs t;
    int64_t ntiles = scan_tiles(n + 1) + 1;
    t.key = b.take<uint32_t>(2 * n);
    t.comp = b.take<int32_t>(n);
    t.nxt = b.take<int32_t>(n);
    t.mn = b.take<int32_t>(n);
    t.flags = b.take<int32_t>(FLAG_WORDS);
    t.size = b.take<int32_t>(n);
    t.heavy_child = b.take<int32_t>(n);
    t.ld = b.take<int32_t>(n);
    t.gpre = b.take<int32_t>(n);
    t.seq = b.take<int32_t>(n);
    t.best = b.take<uint64_t>(n);
    t.pr = b.take<uint64_t>(4 * n);
    t.rootval = b.take<uint64_t>(n);
    t.tourval = b.take<uint64_t>(2 * n);
    t.partial64 = b.take<uint64_t>(scan_tiles(4 * n) + 1);
    t.intree = b.take<uint8_t>(2 * n);
    t.adj = b.take<uint8_t>(n);
    t.partial32 = b.take<int32_t>(scan_tiles(256 * ntiles) + 1);
    t.hist = b.take<int32_t>(256 * ntiles);
    t.sortA = b.take<int32_t>(n);
    t.sortB = b.take<int32_t>(n);
    t.cnt = b.take<int32_t>(n + 1);
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
    k_count_hist<NB><<<(unsigned)ntiles, kBlock, 0, st>>>(src, n, key, hist, ntiles);
    device_scan<int32_t>(hist, hist, (int64_t)NB * ntiles, partial32, nullptr, false, st);
    k_count_scatter<NB, NBITS><<<(unsigned)ntiles, kBlock, 0, st>>>(src, n, key, hist, ntiles, dst,
                                                                    pos_of);
}

void launch_build_tree(const float *img, const LevelGeom &g, const int32_t *plo,
                       const int32_t *phi, int max_width, int width, const hdp_forest &f,
                       void *ws, hipStream_t st) {
    int64_t n = g.off[g.n_pairs];
    size_t bytes;
    TreeWs t = carve_tree_ws(ws, n, &bytes);
    const float4 *im = reinterpret_cast<const float4 *>(img);
    unsigned gn = grid_for(n), gn4 = grid_for(4 * n);

    // 1-2: keys and Boruvka
    k_info_clear<<<1, 64, 0, st>>>(f.info);
    k_bv_init<<<grid_for(n > FLAG_WORDS ? n : FLAG_WORDS), kBlock, 0, st>>>(
        t.comp, t.nxt, t.best, t.mn, t.intree, n, t.flags, f.info);
    k_edge_keys<<<gn, kBlock, 0, st>>>(im, g, plo, phi, max_width, t.key, f.info);
    int bv_rounds = ceil_log2(n) + 2;
    if (bv_rounds > 63) bv_rounds = 63;
    for (int r = 0; r < bv_rounds; ++r) {
        k_bv_minedge<<<gn, kBlock, 0, st>>>(r, t.flags, g, t.key, t.comp, t.best);
        k_bv_hook<<<gn, kBlock, 0, st>>>(r, t.flags, g, t.best, t.comp, t.nxt, t.intree);
        k_bv_compress<<<gn, kBlock, 0, st>>>(r, t.flags, t.comp, t.nxt, t.best, n, f.info);
    }
    // 3: roots
    k_rootmin<<<gn, kBlock, 0, st>>>(t.comp, t.mn, n);
    k_set_tree<<<gn, kBlock, 0, st>>>(t.comp, t.mn, t.intree, g, f.tree, t.adj, f.info);
    // 4: Euler tour ranks
    k_euler_init<<<gn4, kBlock, 0, st>>>(g, t.adj, f.tree, t.pr);
    int rk_rounds = ceil_log2(2 * n) + 2;
    if (rk_rounds > 63) rk_rounds = 63;
    for (int r = 0; r < rk_rounds; ++r) k_rank_round<<<gn4, kBlock, 0, st>>>(r, t.flags, t.pr, 4 * n);
    k_parent<<<gn, kBlock, 0, st>>>(g, t.intree, im, t.pr, f.parent, t.size, f.wgt);
    k_root_info<<<gn, kBlock, 0, st>>>(n, f.tree, t.adj, t.pr, f.parent, t.size, f.wgt, t.rootval);
    // 5: heavy child
    k_heavy<<<gn, kBlock, 0, st>>>(g, t.adj, f.parent, t.size, t.heavy_child);
    // 6: tour offsets, tour values, prefix sum, per-node depth / light depth / preorder
    device_scan<uint64_t>(t.rootval, t.rootval, n, t.partial64, nullptr, false, st);
    k_tour_scatter<<<gn4, kBlock, 0, st>>>(g, t.adj, f.tree, f.parent, t.size, t.heavy_child, t.pr,
                                           t.rootval, t.tourval, f.info);
    int64_t tour_len = 2 * n;  // upper bound; entries past the real length are never read
    device_scan<uint64_t>(t.tourval, t.tourval, tour_len, t.partial64, nullptr, true, st);
    k_node_order<<<gn, kBlock, 0, st>>>(g, t.adj, f.tree, f.parent, t.pr, t.rootval, t.size,
                                        t.tourval, f.depth, t.ld, t.gpre, f.info);
    // 7: rows (stable partition of the preorder by light depth)
    k_scatter_seq<<<gn, kBlock, 0, st>>>(t.gpre, t.seq, n, f.info);
    {
        int64_t ntiles = scan_tiles(n);
        if (ntiles < 1) ntiles = 1;
        LdKey key{t.ld};
        k_count_hist<64><<<(unsigned)ntiles, kBlock, 0, st>>>(t.seq, n, key, t.hist, ntiles);
        device_scan<int32_t>(t.hist, t.hist, 64 * ntiles, t.partial32, nullptr, false, st);
        k_phase_ptr<<<1, 64, 0, st>>>(t.hist, ntiles, n, f.phase_ptr, f.info);
        k_count_scatter<64, 6><<<(unsigned)ntiles, kBlock, 0, st>>>(t.seq, n, key, t.hist, ntiles,
                                                                    f.node, f.row);
    }
    k_rows<<<gn, kBlock, 0, st>>>(g, f.node, f.row, f.parent, f.wgt, t.heavy_child, t.adj, f.prow,
                                  f.heavy, f.lc, f.rw);
    k_intervals<<<gn, kBlock, 0, st>>>(g, plo, phi, f.lo, f.hi);
    // 8: level order (stable LSD radix sort of ids by depth) and level_ptr
    k_iota<<<gn, kBlock, 0, st>>>(t.sortA, n);
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
    k_finish_info<<<1, 64, 0, st>>>(t.flags, f.info, width);
}

}  // namespace hdp
