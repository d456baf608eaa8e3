// Internal declarations shared by the translation units of libara.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "ara.h"

namespace ara {

// Layout constants of the prepared YET and the occurrence tables.
constexpr int kRangeBits = 15;                 // catalogue range of one packed entry
constexpr int kRange = 1 << kRangeBits;
constexpr int kGroups = 16;                    // trial groups per block = wavefronts per workgroup
constexpr int kMaxTrialsPerGroup = 256;
constexpr int kMaxTrialsPerBlock = kGroups * kMaxTrialsPerGroup;   // 4096
constexpr int kSrBits = 16;                    // one occurrence-table "super-range" = 2 ranges
constexpr int kSr = 1 << kSrBits;
constexpr int kSrWords = kSr / 32;             // 2048 bitmap words per super-range
constexpr int kWave = 64;
// Skip codes (0xFFFF) stored after the last code of a prepared YET: one
// 8-byte load per lane of a wavefront reads them in place of codes past a
// segment's end.
constexpr int kPadCodes = 4 * kWave;
// Largest trial a YET prepared with positions holds: a position is 16 bits.
constexpr int64_t kMaxPositions = 65536;
constexpr uint32_t kPrepFlags = ARA_PREP_TRANSPOSED | ARA_PREP_TRIAL_MAJOR | ARA_PREP_POSITIONS;
// Trial slices of the event-major YET copy: one per XCD of the MI355X, so
// that a backward workgroup's gathers of per-trial weights stay in the L2 of
// the XCD it runs on (workgroups are dealt to the XCDs round-robin).
constexpr int kSlices = 8;
// XCDs of the MI355X: consecutive workgroup indexes go to the XCDs in turn.
constexpr int kXcds = 8;
// Devices the library keeps per-device state for.
constexpr int kMaxDevices = 64;

// Error word kept at the head of every workspace.
struct WsHeader {
    int32_t error;          // first device-side error (ARA_E_*), 0 if none
    int32_t pad[63];
};
constexpr size_t kWsHeaderBytes = 256;

void set_error(const std::string &msg);
int32_t fail(int32_t status, const std::string &msg);
int32_t hip_fail(hipError_t e, const char *what);

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

#define ARA_HIP(call)                                              \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return ::ara::hip_fail(_e, #call);   \
    } while (0)

// Carve a caller buffer into 256-byte aligned pieces.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        T *p = reinterpret_cast<T *>(base + used);
        used = align256(used + count * sizeof(T));
        return p;
    }
    size_t bytes() const { return used; }
};

int device_cu_count();

// Host image of the small arrays at the head of a workspace (error header,
// layer lists, table descriptors, work items), laid out at the offsets the
// device carving uses and sent in one host-to-device copy, which also clears
// the error header: one transfer per call instead of one per array.
class HeadImage {
   public:
    explicit HeadImage(void *ws) : ws_(static_cast<char *>(ws)) {}
    template <class T>
    void put(const T *dev_dst, const T *src, size_t n) {
        const size_t off = static_cast<size_t>(reinterpret_cast<const char *>(dev_dst) - ws_);
        grow(off + n * sizeof(T));
        if (n) std::memcpy(buf_.data() + off, src, n * sizeof(T));
    }
    void cover(const void *dev_end) { grow(static_cast<size_t>(static_cast<const char *>(dev_end) - ws_)); }
    int32_t send(hipStream_t st) {
        if (buf_.empty()) return ARA_OK;
        ARA_HIP(hipMemcpyAsync(ws_, buf_.data(), buf_.size(), hipMemcpyHostToDevice, st));
        return ARA_OK;
    }

   private:
    void grow(size_t n) {
        if (buf_.size() < n) buf_.resize(n, 0);
    }
    char *ws_;
    std::vector<unsigned char> buf_;
};

// One YLT row of a metrics launch (the quote server's quotes that finish in
// one iteration share a launch): its values, its results (AAL, PML, TVaR),
// its weights ([3] rows wstride apart, or none), its length and rank, and
// the pieces of its metrics workspace.
struct MetRow {
    const double *ylt;
    double *out;
    double *w;
    int64_t wstride, n, r;
    int32_t nwg, pad;
    uint32_t *hist;    // [2][2048]
    void *st, *part;   // the row's selection state and per-workgroup partials
    uint64_t *cand;    // [n]
};
// The row over a workspace of ara_metrics_workspace_bytes(1, n) bytes.
MetRow metrics_row(void *ws, const double *ylt, int64_t n, double p, double *out, double *w);
// The metrics (and the weights of the rows that have them) of the n_rows
// rows listed at d_rows (device memory); their workspaces are cleared here,
// by a kernel.  max_nwg / max_n: the largest nwg and n among the rows.
int32_t metrics_rows(const MetRow *d_rows, int n_rows, int max_nwg, int64_t max_n, bool any_weights, hipStream_t st);

// Records a start/stop HIP event pair around the enclosed launches when
// profiling is enabled (ara_profile_enable); no-op otherwise.
class ProfScope {
   public:
    ProfScope(int kind, hipStream_t st);
    ~ProfScope();

   private:
    int kind_;
    hipStream_t st_;
    hipEvent_t start_ = nullptr;
};

// Forward/backward occurrence-table workspace layout for one call.
struct OccLayout {
    int n_sr;               // super-ranges
    size_t br_bytes, vals_bytes, cnt_bytes;
};

}  // namespace ara
