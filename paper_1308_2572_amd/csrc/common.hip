// Status strings, thread-local error detail and small shared host helpers.
#include "ara_internal.h"

#include <cstdio>

namespace ara {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int32_t fail(int32_t status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int32_t hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return ARA_E_HIP;
}

int device_cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

}  // namespace ara

extern "C" {

const char *ara_status_string(int32_t status) {
    switch (status) {
        case ARA_OK: return "ok";
        case ARA_E_INVAL: return "invalid argument";
        case ARA_E_RANGE: return "value out of range";
        case ARA_E_DUP: return "duplicate event in one ELT";
        case ARA_E_NOSPACE: return "buffer too small";
        case ARA_E_HIP: return "HIP runtime error";
        case ARA_E_LIMIT: return "implementation limit exceeded";
        default: return "unknown status";
    }
}

const char *ara_last_error(void) { return ara::g_last_error.c_str(); }

int32_t ara_abi_version(void) { return ARA_ABI_VERSION; }

int32_t ara_check_device_error(const void *ws, void *stream) {
    if (!ws) return ara::fail(ARA_E_INVAL, "ara_check_device_error: null workspace");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t err = 0;
    ARA_HIP(hipMemcpyAsync(&err, ws, sizeof(err), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    if (err != 0) {
        return ara::fail(err, std::string("device-side check failed: ") + ara_status_string(err));
    }
    return ARA_OK;
}

}  // extern "C"
