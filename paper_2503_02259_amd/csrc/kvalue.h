// Kernel values on pre-scaled squared distances, shared by the MatVec kernels.
//
// The coordinates are pre-scaled so that the kernel value needs no further
// multiply:
//   FP32 Gaussian   x̃ = x·√(log₂e / (2l²))  →  k = exp2(−‖Δx̃‖²)
//   FP32 Matérn-3/2 x̃ = x·√3 / l            →  a = ‖Δx̃‖, k = (1 + a)·exp2(−a·log₂e)
//   FP64 Gaussian   x̂ = x / (√2·l)          →  k = exp(−‖Δx̂‖²)
//   FP64 Matérn-3/2 x̃ = x·√3 / l            →  a = ‖Δx̃‖, k = (1 + a)·exp(−a)
// With GRAD the second value kg is proportional to ∂k/∂l:
//   Gaussian: ∂k/∂l = k·r²/l³ = kg·(2/(l·log₂e)) (FP32) or kg·(2/l) (FP64), kg = k·r̃²
//   Matérn:   ∂k/∂l = (3r²/l³)·e^{−√3r/l} = kg / l,  kg = a²·e^{−a}
#pragma once

#include "common.h"

namespace higp {

constexpr float kLog2eF = 1.4426950408889634f;
constexpr double kLog2e = 1.4426950408889634;

template <int KERN, bool GRAD>
__device__ __forceinline__ void kval_f32(float r2, float& kv, float& kg) {
  if constexpr (KERN == HIGP_GAUSSIAN) {
    kv = __builtin_amdgcn_exp2f(-r2);
    if constexpr (GRAD) kg = kv * r2;
  } else {
    const float a = __builtin_amdgcn_sqrtf(r2);
    const float e = __builtin_amdgcn_exp2f(-a * kLog2eF);
    kv = fmaf(a, e, e);  // (1 + a)·e^{−a}
    if constexpr (GRAD) kg = r2 * e;
  }
}

template <int KERN, bool GRAD>
__device__ __forceinline__ void kval_f64(double r2, double& kv, double& kg) {
  if constexpr (KERN == HIGP_GAUSSIAN) {
    kv = exp(-r2);
    if constexpr (GRAD) kg = kv * r2;
  } else {
    const double a = sqrt(r2);
    const double e = exp(-a);
    kv = fma(a, e, e);
    if constexpr (GRAD) kg = r2 * e;
  }
}

// Host-side scalings of the two forms (see the table above).
inline double coord_scale(int kernel, int prec, double l) {
  if (kernel == HIGP_MATERN32) return 1.7320508075688772 / l;
  if (prec == HIGP_FP64) return 1.0 / (1.4142135623730951 * l);
  return __builtin_sqrt(kLog2e / (2.0 * l * l));
}

// ∂k/∂l = dl_factor · kg.
inline double dl_factor(int kernel, int prec, double l) {
  if (kernel == HIGP_MATERN32) return 1.0 / l;
  if (prec == HIGP_FP64) return 2.0 / l;
  return 2.0 / (l * kLog2e);
}

}  // namespace higp
