// Device library of the approximated functions: FP32 values (vertex values
// and the hat-function quadrature) and FP64 second derivatives (the knot
// density of Sec. III-B1).  Gaussian (Sec. VI-A), Lorentzian (Sec. VI-B),
// Bessel J0 (Sec. VI-C), plus two test functions with closed-form knots.
#pragma once

#include <hip/hip_runtime.h>

#include "pwl_internal.h"

namespace pwl {

__device__ inline float f_value32(const FuncDesc& f, float x) {
  switch (f.func) {
    case PWL_F_GAUSSIAN: {
      const float s = f.p32[0], amp = f.p32[1];
      return amp * expf(-(x * x) / (2.0f * s * s));
    }
    case PWL_F_LORENTZIAN: {
      const float u = x / f.p32[0];
      return f.p32[1] / fmaf(u, u, 1.0f);
    }
    case PWL_F_BESSEL_J0:
      return f.p32[0] * j0f(x);
    case PWL_F_POLY: {
      float r = f.p32[PWL_MAX_PARAMS - 1];
      for (int k = PWL_MAX_PARAMS - 2; k >= 0; --k) r = fmaf(r, x, f.p32[k]);
      return r;
    }
    case PWL_F_EXP:
      return f.p32[1] * expf(f.p32[0] * x);
    default:
      return __builtin_nanf("");
  }
}

// f''(x) in FP64, from calculus.
__device__ inline double f_second64(const FuncDesc& f, double x) {
  switch (f.func) {
    case PWL_F_GAUSSIAN: {
      const double s = f.p[0], amp = f.p[1];
      const double s2 = s * s;
      return amp * ((x * x) / (s2 * s2) - 1.0 / s2) * exp(-(x * x) / (2.0 * s2));
    }
    case PWL_F_LORENTZIAN: {
      const double g = f.p[0], amp = f.p[1];
      const double u = x / g;
      const double q = 1.0 + u * u;
      return amp * (6.0 * u * u - 2.0) / (g * g * q * q * q);
    }
    case PWL_F_BESSEL_J0: {
      // Bessel's equation gives J0'' = -J0 - J0'/x = J1(x)/x - J0(x); J0''(0) = -1/2.
      const double amp = f.p[0];
      if (x == 0.0) return -0.5 * amp;
      return amp * (j1(x) / x - j0(x));
    }
    case PWL_F_POLY: {
      double r = 0.0;
      for (int k = PWL_MAX_PARAMS - 1; k >= 2; --k) r = fma(r, x, (double)(k * (k - 1)) * f.p[k]);
      return r;
    }
    case PWL_F_EXP: {
      const double al = f.p[0];
      return f.p[1] * al * al * exp(al * x);
    }
    default:
      return __builtin_nan("");
  }
}

// Local knot density |f''|^(2/5) (Sec. III-B1), as 2^(0.4 log2 |f''|)
// (0 at a zero of f'').
__device__ inline double knot_density(const FuncDesc& f, double x) {
  return exp2(0.4 * log2(fabs(f_second64(f, x))));
}

}  // namespace pwl
