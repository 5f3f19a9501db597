// dm_match_images_noalloc: dm_match_images for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation).  Its workspace is a static device array of
// DM_NOALLOC_MAX_BYTES that every GPU holds from the library's code object
// load until the process ends; the call itself allocates nothing.
#include <mutex>

#include "dm_internal.h"

namespace {

// The device array.  In host code this name is a host-side stand-in, not a
// device address: every host use goes through the per-device address below.
static __device__ __align__(256) unsigned char scratch[DM_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
dm_status scratch_address(void** out) {
    int dev = 0;
    dm_status st = dm::check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != DM_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return dm::fail(DM_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        st = dm::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st != DM_OK) return st;
        if (!p) return dm::fail(DM_ERR_HIP, "hipGetSymbolAddress returned a null address");
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return DM_OK;
}

}  // namespace

extern "C" {

dm_status dm_match_images_noalloc(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2,
                                  int ld2, const dm_params* prm, dm_match* out, int capacity, int* n_out,
                                  hipStream_t stream) {
    dm::clear_error();
    dm_plan_info pi;
    dm_status st = dm::plan_pair(prm, W1, H1, W2, H2, &pi);
    if (st != DM_OK) return st;
    if (pi.workspace_bytes > DM_NOALLOC_MAX_BYTES)
        return dm::fail(DM_ERR_WORKSPACE, "the pair needs %llu workspace bytes, above the %llu of the static array",
                        (unsigned long long)pi.workspace_bytes, (unsigned long long)DM_NOALLOC_MAX_BYTES);
    void* ws = nullptr;
    if ((st = scratch_address(&ws)) != DM_OK) return st;
    // Timing records would create events: none are recorded for this call.
    dm::timing_suppress(true);
    st = dm::match_images(img1, W1, H1, ld1, img2, W2, H2, ld2, prm, ws, DM_NOALLOC_MAX_BYTES, out, capacity, n_out,
                          stream);
    dm::timing_suppress(false);
    return st;
}

}  // extern "C"
