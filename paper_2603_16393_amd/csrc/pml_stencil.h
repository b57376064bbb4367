// First differences of the PML sweeps (wave_pml.hip, wave_pml_hbm.hip): the
// 8th-order central first derivative whose weights d_k = (4/5, -1/5, 4/105,
// -1/280) come with the standard 8th-order second difference.  Both sweeps
// evaluate it from this one definition, in translation units compiled
// without implicit multiply-add fusing, so they round alike.
#pragma once

#include "fwi_internal.h"

#pragma clang fp contract(off)

namespace fwi {

constexpr float kD1 = 4.0f / 5.0f;
constexpr float kD2 = -1.0f / 5.0f;
constexpr float kD3 = 4.0f / 105.0f;
constexpr float kD4 = -1.0f / 280.0f;

// Central first difference sum_k d_k (f(+k s) - f(-k s)) at c (unscaled).
__device__ __forceinline__ float dfirst(const float* c, int s) {
    return fmaf(kD1, c[s] - c[-s], fmaf(kD2, c[2 * s] - c[-2 * s], fmaf(kD3, c[3 * s] - c[-3 * s], kD4 * (c[4 * s] - c[-4 * s]))));
}

}  // namespace fwi
