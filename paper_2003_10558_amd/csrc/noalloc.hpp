// vsr_render_noalloc: the fused single-view renderer (vsr_render) with its
// list scratch in a library-held device array instead of a caller buffer,
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array lives in the code object: every GPU that loads the library holds
// its own copy (kNoAllocScratchBytes) until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address is looked up once per device
// with hipGetSymbolAddress and kept in noalloc_ptr[device].
//
// The fused kernel writes each tile's sorted list into its slot of the
// scratch before it reads it back, within the same workgroup, so nothing in
// the array has to start at zero.  Every call on one GPU shares that GPU's
// array: calls that overlap in time on one GPU (two streams, two threads)
// race on it and may give wrong images.
#pragma once
#include <mutex>

#include "api.hpp"

namespace vsr {

constexpr int64_t kNoAllocScratchBytes = int64_t(128) << 20;  // 32,768 tiles of 8x8 pixels: up to 1920x1080
static_assert(kNoAllocScratchBytes == int64_t(VSR_NOALLOC_MAX_TILES) * kFusedCap * 4,
              "the header's tile limit matches the scratch size");

static __device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / 4];

constexpr int kNoAllocMaxDevices = 64;
static void* noalloc_ptr[kNoAllocMaxDevices];
static std::mutex noalloc_mu;

// Device address of this device's scratch array (looked up on the first call
// on a device, with that device current).  VSR_OK or an error code.
static int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "vsr_render_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(VSR_E_ARG, "device %d outside 0..%d", dev, kNoAllocMaxDevices - 1);
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "vsr_render_noalloc: hipGetSymbolAddress");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
            return fail(VSR_E_HIP, "vsr_render_noalloc: scratch array at a NULL or misaligned address");
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return VSR_OK;
}

}  // namespace vsr

extern "C" {

int vsr_render_noalloc(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                       uint32_t* tri_id, float* depth, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !tri_id || !depth || !aligned(map) || !aligned(setup))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(tri_id) & 3u) || (reinterpret_cast<uintptr_t>(depth) & 3u))
        return fail(VSR_E_ARG, "output not 4-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    const int64_t need = fused_scratch_bytes(v->width, v->height);
    if (need > kNoAllocScratchBytes)
        return fail(VSR_E_SPACE, "vsr_render_noalloc: a %dx%d view needs %lld scratch bytes, the library holds %lld "
                    "(at most %d tiles of 8x8 pixels)", v->width, v->height, (long long)need,
                    (long long)kNoAllocScratchBytes, VSR_NOALLOC_MAX_TILES);
    void* scr = nullptr;
    rc = noalloc_scratch(&scr);
    if (rc != VSR_OK) return rc;
    return hip_status(launch_fused(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, scr, tri_id, depth,
                                   hipStream_t(stream)),
                      "vsr_render_noalloc");
}

}  // extern "C"
