// Device library of the approximated functions: FP32 values (vertex values
// and the hat-function quadrature) and FP64 second derivatives (the knot
// density of Sec. III-B1).  Gaussian (Sec. VI-A), Lorentzian (Sec. VI-B),
// Bessel J0 (Sec. VI-C), two test functions with closed-form knots, and any
// f given by samples of f and f'' (the method applies to any continuous f).
#pragma once

#include <hip/hip_runtime.h>

#include "pwl_internal.h"

namespace pwl {

// A sampled f: the cubic spline with values f_i and second derivatives f''_i
// at t_i.  On [t_i, t_{i+1}], u = (x - t_i) / h:
//   f(x)   = (1-u) f_i + u f_{i+1} - h^2 u (1-u) ((2-u) f''_i + (1+u) f''_{i+1}) / 6,
//   f''(x) = (1-u) f''_i + u f''_{i+1};
// outside [t_0, t_S] the end intervals extend.
__device__ inline int sample_cell(const FuncDesc& f, double x, double* u) {
  const double s = (x - f.s_a) / f.s_h;
  double c = floor(s);
  c = fmin(fmax(c, 0.0), (double)(f.S - 1));
  *u = s - c;
  return (int)c;
}

__device__ inline double sampled_value(const FuncDesc& f, double x) {
  double u;
  const int i = sample_cell(f, x, &u);
  const double w = u * (1.0 - u) * f.s_h * f.s_h / 6.0;
  return (1.0 - u) * f.sf[i] + u * f.sf[i + 1] - w * ((2.0 - u) * f.sf2[i] + (1.0 + u) * f.sf2[i + 1]);
}

__device__ inline double sampled_second(const FuncDesc& f, double x) {
  double u;
  const int i = sample_cell(f, x, &u);
  return (1.0 - u) * f.sf2[i] + u * f.sf2[i + 1];
}

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
    case PWL_F_SAMPLED:
      return (float)sampled_value(f, (double)x);
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
    case PWL_F_SAMPLED:
      return sampled_second(f, x);
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
