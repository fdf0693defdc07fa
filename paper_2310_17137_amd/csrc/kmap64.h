// FP64 kernel map shared by the FP64-tile update and the FP64 true residual:
// k = s * map(r^2) with r^2 the ARD squared distance (exact differencing).
#pragma once

#include "ap_internal.h"

namespace ap {

template <int KERN>
__device__ __forceinline__ double kernel_fp64(double r2, double s) {
  if constexpr (KERN == 0) {
    return s * exp(-0.5 * r2);
  } else if constexpr (KERN == 1) {
    const double t = 1.7320508075688772 * sqrt(r2);
    return s * (1.0 + t) * exp(-t);
  } else {
    const double r = sqrt(r2), t = 2.23606797749979 * r;
    return s * (1.0 + t + (5.0 / 3.0) * r2) * exp(-t);
  }
}

}  // namespace ap
