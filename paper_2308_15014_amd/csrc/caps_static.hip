// Search without device allocation: caps_search_static runs the search of
// caps_search in a workspace that lives in the library's own device memory,
// a file-scope array of fixed size that each GPU the library runs on keeps
// until the process ends.  For callers that cannot allocate (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// In host code the array's name stands for a host-side shadow, not for its
// device address: the address is fetched once per device with
// hipGetSymbolAddress (with that device current) and kept; only that
// pointer is passed to kernels.
#include <mutex>

#include "caps_internal.h"

namespace caps {

constexpr size_t kStaticScratchBytes = (size_t)CAPS_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

static std::mutex g_static_mu;
static void *g_static_ptr[kMaxDevices];

// Device address of `scratch` on device `dev` (the current device).
static caps_status static_workspace(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("caps_search_static: device %d outside the supported range", dev);
        return CAPS_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("caps_search_static: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return CAPS_EDEVICE;
        }
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return CAPS_OK;
}

}  // namespace caps

using namespace caps;

extern "C" caps_status caps_search_static(const caps_index *idx, const caps_search_params *sp, const float *q,
                                          int32_t n_q, const int32_t *con_off, const int32_t *con_attr,
                                          const int32_t *con_val, int32_t n_con, int32_t *out_ids, float *out_dist,
                                          int32_t *out_ncand, int32_t *out_nsurv, void *stream) {
    caps_status s = caps_search_check(idx, sp, q, n_q, con_off, con_attr, con_val, n_con);
    if (s != CAPS_OK) return s;
    if (n_q > 0 && (!out_ids || !out_dist)) {
        set_error("caps_search_static: null outputs");
        return CAPS_EINVAL;
    }
    if (sp->workspace_bytes > (int64_t)kStaticScratchBytes) {
        set_error("caps_search_static: workspace_bytes %lld above the static workspace of %zu bytes",
                  (long long)sp->workspace_bytes, kStaticScratchBytes);
        return CAPS_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != idx->ix.device) {
        set_error("caps_search_static: the index's device (%d) must be the current device (%d)", idx->ix.device, dev);
        return CAPS_EINVAL;
    }
    void *ws = nullptr;
    s = static_workspace(dev, &ws);
    if (s != CAPS_OK) return s;
    SearchExtra ex;
    ex.ws = ws;
    ex.ws_bytes = sp->workspace_bytes > 0 ? (size_t)sp->workspace_bytes : kStaticScratchBytes;
    return search(&idx->ix, sp, q, n_q, con_off, con_attr, con_val, n_con, out_ids, out_dist, out_ncand, out_nsurv,
                  nullptr, nullptr, (hipStream_t)stream, &ex);
}
