// The forward for callers that cannot allocate device memory: the same
// kernels as ara_ylt_forward over a workspace the library holds per device.
#include "occ.h"

#include <mutex>
#include <string>

namespace ara {

// The workspace of ara_ylt_forward_noalloc: one array per device, held by
// the library from the first call on that device until the process ends.
// Host code never passes the array's name to a kernel (on the host it names
// a stand-in, not device memory): it uses the device address that
// hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) unsigned char scratch[ARA_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int32_t scratch_address(void **out) {
    int dev = 0;
    ARA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ARA_E_LIMIT, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        ARA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ARA_E_HIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ARA_OK;
}

// *dst = (src ? *src : 0): the call's device-side status, written by a
// kernel so that the variant that allocates nothing also records no memset.
__global__ void k_put_status(int32_t *dst, const int32_t *src) {
    if (threadIdx.x == 0) *dst = src ? *src : 0;
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_ylt_forward_noalloc(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                           const double *elt_terms, const double *layer_terms, int64_t trial_begin,
                                           int64_t trial_end, uint32_t flags, double *ylt, double *s_pre,
                                           int32_t *hits, int32_t *dev_status, void *stream) {
    size_t need = 0;
    int32_t rc = forward_args(tables, yet, layers, elt_terms, layer_terms, trial_begin, trial_end, flags, ylt, hits,
                              &need);
    if (rc) return rc;
    if (need > ARA_NOALLOC_SCRATCH_BYTES)
        return fail(ARA_E_LIMIT, "forward needs " + std::to_string(need) + " bytes of workspace, beyond the " +
                                     std::to_string(static_cast<size_t>(ARA_NOALLOC_SCRATCH_BYTES)) +
                                     " bytes of the no-allocation scratch");
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool empty = layers->n_layers == 0 || trial_end == trial_begin;
    if (!empty && (rc = forward_run(tables, yet, layers, elt_terms, layer_terms, trial_begin, trial_end, flags, ylt,
                                    s_pre, hits, ws, st)))
        return rc;
    if (dev_status) {
        k_put_status<<<1, 64, 0, st>>>(dev_status, empty ? nullptr : static_cast<const int32_t *>(ws));
        ARA_HIP(hipGetLastError());
    }
    return ARA_OK;
}
