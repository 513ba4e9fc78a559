// sst_detect on the library's own static device scratch, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc): the workspace is a file-scope
// device array of fixed size, one copy per GPU, whose address is looked up
// once per device.  Nothing here allocates; every call on a GPU uses that
// GPU's copy, so calls on one GPU that overlap in time race.
#include "sst_internal.h"
#include "../../include/sst.h"

#include <cstdio>
#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

// The scratch array itself.  In host code `scratch` names a host-side
// stand-in, not device memory: only the address returned by
// hipGetSymbolAddress (per device) is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on the first call on
// the device, with that device current), or nullptr with the error set.
void* scratch_of_current_device(int* rc) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *rc = sst::set_error(SST_E_DEVICE, "no usable current HIP device for the static scratch");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[256];
            snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            *rc = sst::set_error(SST_E_DEVICE, msg);
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t sst_noalloc_scratch_bytes(void) { return kScratchBytes; }

int sst_detect_noalloc(const void* frames, int dtype, const float* scale, int n, int h, int w, const double* t,
                       double t_ref, const double* vx, int nvx, const double* vy, int nvy, float threshold,
                       int min_coverage, int k_max, sst_candidate* cand, int32_t* count, double* frame_stats,
                       void* stream) {
    // size first: a problem larger than the scratch is rejected before any
    // device work (sst_workspace_bytes validates the arguments as well)
    const size_t need = sst_workspace_bytes(SST_OP_DETECT, n, h, w, t, t_ref, vx, nvx, vy, nvy, k_max);
    if (need == 0)  // an argument error: the full call reports it (and enqueues nothing)
        return sst::detect_call(frames, dtype, scale, n, h, w, t, t_ref, vx, nvx, vy, nvy, threshold, min_coverage,
                                k_max, cand, count, frame_stats, nullptr, 0, stream, false);
    if (need > kScratchBytes) {
        char msg[256];
        snprintf(msg, sizeof msg, "problem needs %zu bytes of workspace; the static scratch holds %zu", need,
                 kScratchBytes);
        return sst::set_error(SST_E_WORKSPACE, msg);
    }
    int rc = SST_OK;
    void* ws = scratch_of_current_device(&rc);
    if (!ws) return rc;
    return sst::detect_call(frames, dtype, scale, n, h, w, t, t_ref, vx, nvx, vy, nvy, threshold, min_coverage, k_max,
                            cand, count, frame_stats, ws, kScratchBytes, stream, false);
}

}  // extern "C"
