// Backward (placeholder until the adjoint kernels land).
#include "ara_internal.h"

using namespace ara;

extern "C" int32_t ara_ylt_backward_workspace_bytes(const ara_tables *, const ara_yet *, const ara_layers *, int32_t,
                                                    size_t *bytes) {
    if (bytes) *bytes = 0;
    return fail(ARA_E_LIMIT, "backward not available in this build");
}

extern "C" int32_t ara_ylt_backward(const ara_tables *, const ara_yet *, const ara_layers *, const double *,
                                    const double *, int64_t, int64_t, const double *, int32_t, const double *, double *,
                                    double *, void *, size_t, void *) {
    return fail(ARA_E_LIMIT, "backward not available in this build");
}
