// Wavefront-wide operations on binary64 values by DPP (data-parallel
// primitives move values between lanes inside the VALU: no LDS traffic).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ara {

// Cross-lane move of a binary64 value: CTRL is the DPP control; lanes whose
// source is outside the pattern (or whose row is masked off) read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) |
                                                       static_cast<uint32_t>(lo)));
}

// Inclusive prefix sum over the 64 lanes: shifts of 1, 2, 4, 8 inside each
// row of 16 lanes, then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then the first two rows' total into rows 2 and 3
// (row_bcast:31).  Lane 63 ends with the sum of all lanes, in a fixed order.
__device__ __forceinline__ double wave_inclusive_sum(double x) {
    x += dpp_f64<0x111, 0xf>(x);   // row_shr:1
    x += dpp_f64<0x112, 0xf>(x);   // row_shr:2
    x += dpp_f64<0x114, 0xf>(x);   // row_shr:4
    x += dpp_f64<0x118, 0xf>(x);   // row_shr:8
    x += dpp_f64<0x142, 0xa>(x);   // row_bcast:15
    x += dpp_f64<0x143, 0xc>(x);   // row_bcast:31
    return x;
}

// Lane 63's value, in every lane.
__device__ __forceinline__ double lane63(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(b), 63);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(b >> 32), 63);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

}  // namespace ara
