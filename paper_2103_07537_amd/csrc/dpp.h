// Wavefront reductions by DPP moves (no LDS) shared by the kernel files.
#pragma once

#include "common.h"

namespace mbamg {

// v from the lane selected by the DPP control CTRL within the 16-lane rows of
// ROWMASK; 0 where that lane is outside the row or the row is masked
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_in(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, true));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_in(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of G lanes (4, 8, 16 or 64), valid in the
// group's last lane: the row shifts by 1, 2, 4 and 8 only ever add lanes of
// the same group into that lane; for G = 64 the row broadcasts 15 and 31 then
// add the four rows up in lane 63.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 64, "group of 4, 8, 16 or 64 lanes");
    v += dpp_in<0x111, 0xF>(v);                          // row_shr:1
    v += dpp_in<0x112, 0xF>(v);                          // row_shr:2
    if constexpr (G >= 8) v += dpp_in<0x114, 0xF>(v);    // row_shr:4
    if constexpr (G >= 16) v += dpp_in<0x118, 0xF>(v);   // row_shr:8
    if constexpr (G == 64) {
        v += dpp_in<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
        v += dpp_in<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    }
    return v;
}

}  // namespace mbamg
