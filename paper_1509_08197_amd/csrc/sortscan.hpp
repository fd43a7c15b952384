// Device-wide prefix scans and stable counting sorts used by the tree builder.
// Deterministic (integer arithmetic only), no memsets, fixed launch shapes.
#pragma once

#include "common.hpp"

namespace hdp {

constexpr int kScanPerThread = 4;
constexpr int kScanTile = kBlock * kScanPerThread;  // 1024 elements per workgroup

__device__ __forceinline__ uint64_t lanemask_lt() {
    int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan of one value per lane across a 64-wide wavefront.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread across a workgroup of NT threads.
// Returns the exclusive prefix; *total receives the workgroup sum.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan_n(T x, T *total) {
    __shared__ T wsum[NT / 64];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T inc = wave_incl_scan(x);
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T s = wsum[w];
        if (w < wv) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *total) {
    return block_excl_scan_n<kBlock>(x, total);
}

// Scan inputs may be stored narrower than the sums: wide(x) gives the value
// of a stored element (identity by default).
struct WidenSame {
    template <typename X>
    __device__ X operator()(X x) const { return x; }
};

// A thread's kScanPerThread consecutive elements.  A full run is loaded
// without conditions, so that all its loads are in flight together.
template <typename T, typename TIn, typename Widen>
__device__ __forceinline__ void load_run(const TIn *__restrict__ in, int64_t base, int64_t n,
                                         Widen wide, T (&v)[kScanPerThread]) {
    if (base + kScanPerThread <= n) {
        TIn x[kScanPerThread];
#pragma unroll
        for (int i = 0; i < kScanPerThread; ++i) x[i] = in[base + i];
#pragma unroll
        for (int i = 0; i < kScanPerThread; ++i) v[i] = (T)wide(x[i]);
    } else {
#pragma unroll
        for (int i = 0; i < kScanPerThread; ++i) v[i] = base + i < n ? (T)wide(in[base + i]) : (T)0;
    }
}

template <typename T, typename TIn = T, typename Widen = WidenSame>
__global__ void k_scan_reduce(const TIn *__restrict__ in, int64_t n, T *__restrict__ partial,
                              Widen wide = Widen()) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPerThread;
    T v[kScanPerThread];
    load_run(in, base, n, wide, v);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) s += v[i];
    T tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Tile sums are scanned in blocks of kScanTile: every workgroup scans one
// block in place (exclusive) and writes the block's total to sup[block]; a
// tile's offset is then its scanned sum plus the totals of the blocks before
// its own (few: one per kScanTile tiles), summed by its workgroup.
template <typename T>
__global__ void k_scan_partials(T *__restrict__ part, int64_t nb, T *__restrict__ sup) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPerThread;
    T v[kScanPerThread];
    load_run(part, base, nb, WidenSame(), v);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) s += v[i];
    T tot;
    T ex = block_excl_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        if (base + i < nb) part[base + i] = ex;
        ex += v[i];
    }
    if (threadIdx.x == 0) sup[blockIdx.x] = tot;
}

// Sum of sup[0..m) over the workgroup (every thread receives it).
template <typename T>
__device__ __forceinline__ T block_sum_prefix(const T *__restrict__ sup, int64_t m) {
    T a = 0;
    for (int64_t j = threadIdx.x; j < m; j += kBlock) a += sup[j];
    T tot;
    block_excl_scan(a, &tot);
    return tot;
}

// Lists of at most kDirectTiles tile sums are not scanned by a launch of
// their own: every tile sums the unscanned sums before it, kDirectPer loads
// per thread issued together (the sums are a few KB, served from L2).
constexpr int kDirectPer = 16;
constexpr int64_t kDirectTiles = (int64_t)kBlock * kDirectPer;

template <typename T>
__device__ __forceinline__ T block_sum_direct(const T *__restrict__ part, int64_t m) {
    T v[kDirectPer];
#pragma unroll
    for (int i = 0; i < kDirectPer; ++i) {
        const int64_t j = (int64_t)i * kBlock + threadIdx.x;
        v[i] = j < m ? part[j] : (T)0;
    }
    T a = 0;
#pragma unroll
    for (int i = 0; i < kDirectPer; ++i) a += v[i];
    T tot;
    block_excl_scan(a, &tot);
    return tot;
}

// Scan of one tile, offset by its scanned tile sum and the block totals
// before it, or (direct) by the sum of the unscanned tile sums before it.
// grand (may be NULL) receives the total from the last tile.
template <typename T, typename TIn = T, typename Widen = WidenSame>
__global__ void k_scan_apply(const TIn *__restrict__ in, T *__restrict__ out, int64_t n,
                             const T *__restrict__ partial, const T *__restrict__ sup,
                             T *__restrict__ grand, int inclusive, int direct,
                             Widen wide = Widen()) {
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kScanTile + threadIdx.x * kScanPerThread;
    T v[kScanPerThread];
    load_run(in, base, n, wide, v);
    const T pre = direct ? block_sum_direct(partial, tile)
                         : partial[tile] + block_sum_prefix(sup, tile / kScanTile);
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) s += v[i];
    T tot;
    T ex = block_excl_scan(s, &tot) + pre;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        T nx = ex + v[i];
        if (base + i < n) out[base + i] = inclusive ? nx : ex;
        ex = nx;
    }
    if (grand && tile == gridDim.x - 1 && threadIdx.x == 0) *grand = pre + tot;
}

inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
// Scratch elements of a scan of n elements: the tile sums, then the block totals.
inline int64_t scan_scratch(int64_t n) {
    const int64_t nb = scan_tiles(n) < 1 ? 1 : scan_tiles(n);
    return nb + scan_tiles(nb) + 1;
}
// Scan of the tile sums part[0..nb) (blockwise; skipped for at most
// kDirectTiles sums, which every tile then adds up itself) and the tiles of
// in.  part is left unscanned in the direct case.
template <typename T, typename TIn, typename Widen>
inline void scan_sums_and_apply(const TIn *in, T *out, int64_t n, T *part, int64_t nb, T *grand,
                                bool inclusive, hipStream_t st, Widen wide) {
    const bool direct = nb <= kDirectTiles;
    if (!direct) {
        const int64_t nsup = scan_tiles(nb);
        k_scan_partials<T><<<(unsigned)nsup, kBlock, 0, st>>>(part, nb, part + nb);
    }
    k_scan_apply<T, TIn, Widen><<<(unsigned)nb, kBlock, 0, st>>>(
        in, out, n, part, part + nb, grand, inclusive ? 1 : 0, direct ? 1 : 0, wide);
}

// out[i] = sum of in[0..i-1] (exclusive) or in[0..i] (inclusive); in == out allowed.
// partial: scratch of scan_scratch(n) elements; grand (device, may be NULL) = total.
// Three launches (two for at most kDirectTiles tiles): per-tile sums, their
// blockwise scan, then every tile's own scan.
template <typename T, typename TIn = T, typename Widen = WidenSame>
inline void device_scan(const TIn *in, T *out, int64_t n, T *partial, T *grand, bool inclusive,
                        hipStream_t st, Widen wide = Widen()) {
    int64_t nb = scan_tiles(n);
    if (nb < 1) nb = 1;
    k_scan_reduce<T, TIn, Widen><<<(unsigned)nb, kBlock, 0, st>>>(in, n, partial, wide);
    scan_sums_and_apply(in, out, n, partial, nb, grand, inclusive, st, wide);
}

// ---------------------------------------------------------------------------
// Tile of this workgroup when the grid (band_grid(ntiles) workgroups) deals
// contiguous bands of tiles to the XCDs, so that neighbouring tiles share an
// L2; -1 past the last tile.
__device__ __forceinline__ int64_t band_tile(int64_t ntiles) {
    const int64_t per = (ntiles + kXcds - 1) / kXcds;
    const int64_t t = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    return t < ntiles ? t : -1;
}
inline unsigned band_grid(int64_t ntiles) {
    return (unsigned)(kXcds * ((ntiles + kXcds - 1) / kXcds));
}

// Stable counting sort of the sequence src[0..n) by a small key (< NB <= 256).
// key_of(i, x) gives the key of element x = src[i].  Histogram per tile of
// 1024 elements (bin-major so that one exclusive scan gives every tile's base),
// then a stable scatter that ranks equal keys with wavefront ballots.

template <int NB, typename KeyFn>
__global__ void k_count_hist(const int32_t *__restrict__ src, int64_t n, KeyFn key_of,
                             int32_t *__restrict__ hist, int64_t ntiles) {
    __shared__ int32_t h[NB];
    const int64_t tile = band_tile(ntiles);
    if (tile < 0) return;
    for (int k = threadIdx.x; k < NB; k += kBlock) h[k] = 0;
    __syncthreads();
    int64_t base = tile * kScanTile;
    // elements, then keys, each one batch of loads
    int32_t xs[kScanPerThread];
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
        const int64_t e = base + q * kBlock + threadIdx.x;
        xs[q] = e < n ? src[e] : 0;
    }
    int ks[kScanPerThread];
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
        const int64_t e = base + q * kBlock + threadIdx.x;
        ks[q] = e < n ? key_of(e, xs[q]) : -1;
    }
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q)
        if (ks[q] >= 0) atomicAdd(&h[ks[q]], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < NB; k += kBlock) hist[(int64_t)k * ntiles + tile] = h[k];
}

template <int NB, int NBITS, typename KeyFn>
__device__ __forceinline__ void count_scatter_tile(const int32_t *__restrict__ src, int64_t n,
                                                   KeyFn key_of, const int32_t *__restrict__ offs,
                                                   int64_t ntiles, int32_t *__restrict__ dst,
                                                   int32_t *__restrict__ pos_of, int64_t tile) {
    __shared__ int32_t run[NB];
    __shared__ int32_t wcnt[kBlock / 64][NB];
    int wv = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < NB; k += kBlock) {
        run[k] = offs[(int64_t)k * ntiles + tile];
        for (int w = 0; w < kBlock / 64; ++w) wcnt[w][k] = 0;
    }
    __syncthreads();
    int64_t base = tile * kScanTile;
    // every step's element and key loaded up front (two batches of loads)
    int32_t xs[kScanPerThread];
    int ks[kScanPerThread];
#pragma unroll
    for (int step = 0; step < kScanPerThread; ++step) {
        const int64_t e = base + step * kBlock + threadIdx.x;
        xs[step] = e < n ? src[e] : 0;
    }
#pragma unroll
    for (int step = 0; step < kScanPerThread; ++step) {
        const int64_t e = base + step * kBlock + threadIdx.x;
        ks[step] = e < n ? key_of(e, xs[step]) : 0;
    }
#pragma unroll
    for (int step = 0; step < kScanPerThread; ++step) {
        int64_t e = base + step * kBlock + threadIdx.x;
        bool valid = e < n;
        int32_t x = xs[step];
        int key = ks[step];
        uint64_t m = __ballot(valid);
        if (!valid) m = ~m;
#pragma unroll
        for (int b = 0; b < NBITS; ++b) {
            bool bit = (key >> b) & 1;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        int rnk = __popcll(m & lanemask_lt());
        if (valid && rnk == 0) wcnt[wv][key] = __popcll(m);
        __syncthreads();
        if (valid) {
            int p = run[key] + rnk;
            for (int w = 0; w < wv; ++w) p += wcnt[w][key];
            dst[p] = x;
            if (pos_of) pos_of[x] = p;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < NB; k += kBlock) {
            int add = 0;
            for (int w = 0; w < kBlock / 64; ++w) { add += wcnt[w][k]; wcnt[w][k] = 0; }
            run[k] += add;
        }
        __syncthreads();
    }
}

template <int NB, int NBITS, typename KeyFn>
__global__ void k_count_scatter(const int32_t *__restrict__ src, int64_t n, KeyFn key_of,
                                const int32_t *__restrict__ offs, int64_t ntiles,
                                int32_t *__restrict__ dst, int32_t *__restrict__ pos_of) {
    const int64_t tile = band_tile(ntiles);
    if (tile < 0) return;
    count_scatter_tile<NB, NBITS>(src, n, key_of, offs, ntiles, dst, pos_of, tile);
}

}  // namespace hdp
