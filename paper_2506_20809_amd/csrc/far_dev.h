// Device helpers of the vector-unit far-field sums.
#pragma once

#include <hip/hip_runtime.h>

namespace sbie {

// 1/sqrt(x): the hardware estimate in FP32; in FP64 the estimate refined by
// two Newton steps y <- y + y (1 - x y^2) / 2.
template <typename R>
__device__ inline R rsq_t(R x);
template <>
__device__ inline float rsq_t<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ inline double rsq_t<double>(double x) {
  double yv = __builtin_amdgcn_rsq(x);
  double e = fma(-x * yv, yv, 1.0);
  yv = fma(0.5 * yv, e, yv);
  e = fma(-x * yv, yv, 1.0);
  return fma(0.5 * yv, e, yv);
}

// acc + v with the rounding error of the addition kept in lo (TwoSum).
template <typename R>
__device__ inline void two_sum_add(R& acc, R& lo, R v) {
  const R sum = acc + v;
  const R bp = sum - acc;
  lo += (acc - (sum - bp)) + (v - bp);
  acc = sum;
}

}  // namespace sbie
