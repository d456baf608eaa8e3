// Status strings, thread-local error detail and small shared host helpers.
#include "ara_internal.h"

#include <cstdio>
#include <mutex>
#include <vector>

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

struct ProfPending {
    int kind;
    hipEvent_t start, stop;
};

static std::mutex g_prof_mu;
static uint32_t g_prof_mask = 0;   // bit k: record kind k
static std::vector<ProfPending> g_prof_pending;
static double g_prof_ms[ARA_PROF_KINDS];
static int64_t g_prof_n[ARA_PROF_KINDS];

ProfScope::ProfScope(int kind, hipStream_t st) : kind_(kind), st_(st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!((g_prof_mask >> kind) & 1u)) return;
    if (hipEventCreate(&start_) != hipSuccess) {
        start_ = nullptr;
        return;
    }
    hipEventRecord(start_, st_);
}

ProfScope::~ProfScope() {
    if (!start_) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess) {
        hipEventDestroy(start_);
        return;
    }
    hipEventRecord(stop, st_);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({kind_, start_, stop});
}

static void prof_drain_locked() {
    for (auto &p : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            g_prof_ms[p.kind] += ms;
            g_prof_n[p.kind] += 1;
        }
        hipEventDestroy(p.start);
        hipEventDestroy(p.stop);
    }
    g_prof_pending.clear();
}

}  // namespace ara

extern "C" {

int32_t ara_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(ara::g_prof_mu);
    ara::g_prof_mask = on ? ((1u << ARA_PROF_KINDS) - 1u) : 0u;
    return ARA_OK;
}

int32_t ara_profile_enable_kinds(uint32_t mask) {
    if (mask >> ARA_PROF_KINDS) return ara::fail(ARA_E_INVAL, "ara_profile_enable_kinds: unknown kind");
    std::lock_guard<std::mutex> lk(ara::g_prof_mu);
    ara::g_prof_mask = mask;
    return ARA_OK;
}

int32_t ara_profile_read(int32_t kind, double *total_ms, int64_t *launches) {
    if (kind < 0 || kind >= ARA_PROF_KINDS) return ara::fail(ARA_E_INVAL, "ara_profile_read: unknown kind");
    std::lock_guard<std::mutex> lk(ara::g_prof_mu);
    ara::prof_drain_locked();
    if (total_ms) *total_ms = ara::g_prof_ms[kind];
    if (launches) *launches = ara::g_prof_n[kind];
    return ARA_OK;
}

int32_t ara_profile_reset(void) {
    std::lock_guard<std::mutex> lk(ara::g_prof_mu);
    ara::prof_drain_locked();
    for (int k = 0; k < ARA_PROF_KINDS; ++k) {
        ara::g_prof_ms[k] = 0.0;
        ara::g_prof_n[k] = 0;
    }
    return ARA_OK;
}

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
