// ELT direct-access tables (Section III): one dense binary32 array per ELT
// over the whole catalogue, 0 for absent events, plus a presence bitmap per
// ELT marking the non-zero entries.
#include "ara_internal.h"

#include <vector>

namespace ara {

static size_t tables_bytes(int32_t n_elts, int32_t catalog) {
    const size_t words = (static_cast<size_t>(catalog) + 31) / 32;
    Carver c(nullptr);
    c.take<float>(static_cast<size_t>(n_elts) * catalog);
    c.take<uint32_t>(static_cast<size_t>(n_elts) * words);
    c.take<int32_t>(64);
    return c.bytes();
}

// Pass 1: range/finiteness checks, duplicate detection through the presence
// bitmap, scatter of the losses.
__global__ void k_tab_scatter(const int64_t *__restrict__ rec_off, const int32_t *__restrict__ rec_ids,
                              const float *__restrict__ rec_loss, int32_t catalog, int32_t words,
                              float *__restrict__ loss, uint32_t *__restrict__ present, int32_t *__restrict__ err) {
    const int k = blockIdx.y;
    const int64_t a = rec_off[k], b = rec_off[k + 1];
    for (int64_t i = a + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < b;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t id = rec_ids[i];
        const float l = rec_loss[i];
        if (id < 0 || id >= catalog) {
            atomicCAS(err, 0, ARA_E_RANGE);
            continue;
        }
        if (!(l >= 0.0f) || !(l <= 3.402823466e38f)) {
            atomicCAS(err, 0, ARA_E_INVAL);
            continue;
        }
        const uint32_t bit = 1u << (id & 31);
        const uint32_t old = atomicOr(&present[static_cast<size_t>(k) * words + (id >> 5)], bit);
        if (old & bit) {
            atomicCAS(err, 0, ARA_E_DUP);
            continue;
        }
        loss[static_cast<size_t>(k) * catalog + id] = l;
    }
}

// Pass 2: records stored with loss 0 are indistinguishable from absence.
__global__ void k_tab_clear_zero(const int64_t *__restrict__ rec_off, const int32_t *__restrict__ rec_ids,
                                 const float *__restrict__ rec_loss, int32_t words, uint32_t *__restrict__ present) {
    const int k = blockIdx.y;
    const int64_t a = rec_off[k], b = rec_off[k + 1];
    for (int64_t i = a + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < b;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (rec_loss[i] == 0.0f) {
            const int32_t id = rec_ids[i];
            atomicAnd(&present[static_cast<size_t>(k) * words + (id >> 5)], ~(1u << (id & 31)));
        }
    }
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_build_elt_tables_bytes(int32_t n_elts, int32_t catalog, size_t *bytes) {
    if (!bytes) return fail(ARA_E_INVAL, "ara_build_elt_tables_bytes: null output");
    if (n_elts < 0 || catalog <= 0) return fail(ARA_E_INVAL, "ara_build_elt_tables_bytes: bad size");
    if (catalog > ARA_MAX_CATALOG) return fail(ARA_E_LIMIT, "catalog exceeds ARA_MAX_CATALOG");
    *bytes = tables_bytes(n_elts, catalog);
    return ARA_OK;
}

extern "C" int32_t ara_build_elt_tables(int32_t n_elts, int32_t catalog, const int64_t *rec_off,
                                        const int32_t *rec_ids, const float *rec_loss, void *buf, size_t buf_bytes,
                                        void *stream, ara_tables *out) {
    if (!rec_off || !buf || !out) return fail(ARA_E_INVAL, "ara_build_elt_tables: null pointer");
    if (n_elts < 0 || catalog <= 0) return fail(ARA_E_INVAL, "ara_build_elt_tables: bad size");
    if (catalog > ARA_MAX_CATALOG) return fail(ARA_E_LIMIT, "catalog exceeds ARA_MAX_CATALOG");
    if (buf_bytes < tables_bytes(n_elts, catalog)) return fail(ARA_E_NOSPACE, "ara_build_elt_tables: buffer too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t words = (catalog + 31) / 32;
    Carver c(buf);
    float *loss = c.take<float>(static_cast<size_t>(n_elts) * catalog);
    uint32_t *present = c.take<uint32_t>(static_cast<size_t>(n_elts) * words);
    int32_t *misc = c.take<int32_t>(64);
    std::vector<int64_t> off(static_cast<size_t>(n_elts) + 1);
    ARA_HIP(hipMemcpyAsync(off.data(), rec_off, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    int64_t max_rec = 0;
    if (off[0] != 0) return fail(ARA_E_RANGE, "rec_off[0] must be 0");
    for (int32_t k = 0; k < n_elts; ++k) {
        if (off[k + 1] < off[k]) return fail(ARA_E_RANGE, "rec_off must be non-decreasing");
        max_rec = std::max<int64_t>(max_rec, off[k + 1] - off[k]);
    }
    if (max_rec > 0 && (!rec_ids || !rec_loss)) return fail(ARA_E_INVAL, "ara_build_elt_tables: null records");
    ARA_HIP(hipMemsetAsync(loss, 0, static_cast<size_t>(n_elts) * catalog * sizeof(float), st));
    ARA_HIP(hipMemsetAsync(present, 0, static_cast<size_t>(n_elts) * words * sizeof(uint32_t), st));
    ARA_HIP(hipMemsetAsync(misc, 0, 64 * sizeof(int32_t), st));
    if (n_elts > 0 && max_rec > 0) {
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((max_rec + 255) / 256, 4096));
        dim3 grid(gx, static_cast<unsigned>(n_elts));
        k_tab_scatter<<<grid, 256, 0, st>>>(rec_off, rec_ids, rec_loss, catalog, words, loss, present, misc);
        ARA_HIP(hipGetLastError());
        int32_t err = 0;
        ARA_HIP(hipMemcpyAsync(&err, misc, sizeof(err), hipMemcpyDeviceToHost, st));
        ARA_HIP(hipStreamSynchronize(st));
        if (err) return fail(err, std::string("ara_build_elt_tables: ") + ara_status_string(err));
        k_tab_clear_zero<<<grid, 256, 0, st>>>(rec_off, rec_ids, rec_loss, words, present);
        ARA_HIP(hipGetLastError());
        ARA_HIP(hipStreamSynchronize(st));
    }
    ara_tables t{};
    t.n_elts = n_elts;
    t.catalog = catalog;
    t.words = words;
    t.loss = loss;
    t.present = present;
    *out = t;
    return ARA_OK;
}
