// hdp_match_layer_noalloc: the matching of one layer (cost, aggregation,
// winner-takes-all) with its scratch space in a fixed device array instead of
// a caller workspace, for callers that cannot allocate device memory.
//
// The array below is a device symbol: in host code its name is only a
// host-side stand-in.  Its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept in g_scratch; every
// launch and copy uses that address, never the symbol's name.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hdp.h"
#include "kernels.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[HDP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once taken

// Device address of this device's copy of the array (taken on first use).
hipError_t scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t hdp_match_layer_noalloc_max_bytes(void) { return (size_t)HDP_NOALLOC_SCRATCH_BYTES; }

hdp_status hdp_match_layer_noalloc(const float *left, const float *right,
                                   const hdp_shape *shapes, int32_t n_pairs,
                                   const hdp_forest *f, int32_t width,
                                   const hdp_cost_params *p, float sigma, float *agg,
                                   int32_t *disp, void *stream) {
    if (!f || f->n < 1 || width < 1 || width > HDP_MAX_LABELS) return HDP_EINVAL;
    // the same scratch layout as the workspace of hdp_match_layer, bounded by the array
    const size_t need = hdp::aggregate_workspace_bytes(f->n, width);
    if (need > (size_t)HDP_NOALLOC_SCRATCH_BYTES) return HDP_EWORKSPACE;
    void *ws = nullptr;
    if (scratch_ptr(&ws) != hipSuccess) return HDP_EHIP;
    // validation of every other argument, then the launches of hdp_match_layer
    return hdp_match_layer(left, right, shapes, n_pairs, f, width, p, sigma, agg, disp, ws,
                           need, stream);
}

}  // extern "C"
