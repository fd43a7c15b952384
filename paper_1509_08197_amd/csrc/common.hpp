// Shared device-side definitions of the HDP library (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hdp.h"

namespace hdp {

constexpr int kBlock = 256;  // threads per workgroup (4 wavefronts of 64)

// Geometry of one pyramid layer of a batch, passed to kernels by value.
struct LevelGeom {
    int32_t n_pairs;
    int32_t level;                    // pyramid layer (edge keys scale by 4^level)
    int32_t off[HDP_MAX_PAIRS + 1];   // first pixel of each pair, off[n_pairs] = n
    int32_t H[HDP_MAX_PAIRS];
    int32_t W[HDP_MAX_PAIRS];
    int32_t dmax[HDP_MAX_PAIRS];
    int32_t toff[HDP_MAX_PAIRS + 1];  // first kTile x kTile tile of each pair (row-major tiles)
};

constexpr int kTile = 32;  // side of the square pixel tiles of the tree builder's local phases

// Pair that holds global pixel v: a binary search for the first active lane's
// pixel, uniform over the wavefront (scalar loads of the offsets), then every
// lane steps to its own pair (no steps when the wavefront's pixels lie in one
// pair).
__device__ __forceinline__ int pair_of(const LevelGeom &g, int v) {
    const int v0 = __builtin_amdgcn_readfirstlane(v);
    int lo = 0, hi = g.n_pairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (g.off[mid] <= v0) lo = mid; else hi = mid - 1;
    }
    while (lo > 0 && g.off[lo] > v) --lo;
    while (lo + 1 < g.n_pairs && g.off[lo + 1] <= v) ++lo;
    return lo;
}

// Element idx of an array of less than 4 GiB, addressed by a 32-bit byte
// offset from the base: the load takes the scalar-base + 32-bit vector-offset
// form (one address register instead of two).  Every per-pixel and per-row
// array of a batch qualifies: a batch holds at most 64 pairs of fewer than
// 2^22 pixels, so fewer than 2^28 elements of at most 16 bytes.
template <typename T>
__device__ __forceinline__ T at32(const T *base, uint32_t idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        (uint64_t)(idx * (uint32_t)sizeof(T)));
}

struct PixelPos {
    int pair, x, y, W, H, base;
};

__device__ __forceinline__ PixelPos pixel_pos(const LevelGeom &g, int v) {
    PixelPos p;
    p.pair = pair_of(g, v);
    p.base = g.off[p.pair];
    p.W = g.W[p.pair];
    p.H = g.H[p.pair];
    int local = v - p.base;
    p.y = local / p.W;
    p.x = local - p.y * p.W;
    return p;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) in turn.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t gtid() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}

// Diagnostic launch timer (HIP events around the launches of one kernel class).
void timer_before(int kernel_class, hipStream_t st);
void timer_after(int kernel_class, hipStream_t st);

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    int64_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace hdp
