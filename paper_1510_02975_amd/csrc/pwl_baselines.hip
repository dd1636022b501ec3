// Baselines beside the table: direct FP32 evaluation of f with the device
// math library (expf / __expf Gaussians - the comparison of Sec. VI-A - and
// every built-in f), and a plain copy, the practical HBM reference and the
// calibration of the traffic counters.  They stream like the evaluators:
// 16-byte non-temporal loads and stores, U vectors per thread in flight.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwl_func.h"
#include "pwl_internal.h"
#include "pwl_stream.h"

namespace pwl {

namespace {

constexpr int kStreamUnroll = 4;    // float4 vectors per thread per iteration (direct kernels)

using stream::v4f;

// Points [4 n4, n) (or all of them when the arrays are not 16-byte aligned,
// n4 = 0) go through this grid-strided scalar loop.
#define PWL_SCALAR_TAIL(...)                                                                \
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;         \
       i += (int64_t)gridDim.x * blockDim.x) {                                              \
    __VA_ARGS__;                                                                            \
  }

template <bool kFast>
__global__ __launch_bounds__(256) void k_direct_gaussian(const float* __restrict__ x,
                                                         float* __restrict__ y, int64_t n4, int64_t n,
                                                         float c, float amp) {
  constexpr int kUnroll = kStreamUnroll;
  // y = amp exp(c x^2) with c = -1 / (2 s^2)
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x);
  v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y);
  const int64_t bs = blockDim.x;
  const int64_t stride = (int64_t)gridDim.x * bs * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * bs * kUnroll + threadIdx.x; base < n4; base += stride) {
    v4f xv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) xv[u] = __builtin_nontemporal_load(x4 + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) {
        v4f yv;
        if (kFast) {
          yv.x = amp * __expf(c * xv[u].x * xv[u].x);
          yv.y = amp * __expf(c * xv[u].y * xv[u].y);
          yv.z = amp * __expf(c * xv[u].z * xv[u].z);
          yv.w = amp * __expf(c * xv[u].w * xv[u].w);
        } else {
          yv.x = amp * expf(c * xv[u].x * xv[u].x);
          yv.y = amp * expf(c * xv[u].y * xv[u].y);
          yv.z = amp * expf(c * xv[u].z * xv[u].z);
          yv.w = amp * expf(c * xv[u].w * xv[u].w);
        }
        __builtin_nontemporal_store(yv, y4 + i);
      }
    }
  }
  PWL_SCALAR_TAIL(y[i] = amp * (kFast ? __expf(c * x[i] * x[i]) : expf(c * x[i] * x[i])))
}

// Direct FP32 evaluation of f at every point, the same streaming shape.
__global__ __launch_bounds__(256) void k_direct_func(FuncDesc f, const float* __restrict__ x,
                                                     float* __restrict__ y, int64_t n4, int64_t n) {
  constexpr int kUnroll = kStreamUnroll;
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x);
  v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y);
  const int64_t bs = blockDim.x;
  const int64_t stride = (int64_t)gridDim.x * bs * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * bs * kUnroll + threadIdx.x; base < n4; base += stride) {
    v4f xv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) xv[u] = __builtin_nontemporal_load(x4 + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) {
        v4f yv;
        yv.x = f_value32(f, xv[u].x);
        yv.y = f_value32(f, xv[u].y);
        yv.z = f_value32(f, xv[u].z);
        yv.w = f_value32(f, xv[u].w);
        __builtin_nontemporal_store(yv, y4 + i);
      }
    }
  }
  PWL_SCALAR_TAIL(y[i] = f_value32(f, x[i]))
}

// The copy reference takes the launch shape that measured fastest for a
// plain copy on MI355X (1024-thread workgroups, 8 vectors per thread, 32
// workgroups per CU; 6.24 TB/s on 2^28 elements against 5.8 for 256-thread
// workgroups and 4 vectors).
constexpr int kCopyUnroll = 8, kCopyBlock = 1024, kCopyWgPerCu = 32;

__global__ __launch_bounds__(kCopyBlock) void k_copy(const float* __restrict__ src, float* __restrict__ dst,
                                                     int64_t n4, int64_t n) {
  constexpr int kUnroll = kCopyUnroll;
  const v4f* __restrict__ s4 = reinterpret_cast<const v4f*>(src);
  v4f* __restrict__ d4 = reinterpret_cast<v4f*>(dst);
  const int64_t bs = blockDim.x;
  const int64_t stride = (int64_t)gridDim.x * bs * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * bs * kUnroll + threadIdx.x; base < n4; base += stride) {
    v4f v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) v[u] = __builtin_nontemporal_load(s4 + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) __builtin_nontemporal_store(v[u], d4 + i);
    }
  }
  PWL_SCALAR_TAIL(dst[i] = src[i])
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

LaunchShape baseline_shape(int64_t n4, int64_t n, int num_cu) {
  const int block = 256;
  const int64_t work = (n4 > 0) ? (n4 + block * kStreamUnroll - 1) / (block * kStreamUnroll)
                                : (n + block - 1) / block;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * 8, work));
  return LaunchShape{block, grid, 0};
}

}  // namespace

hipError_t launch_direct_gaussian(const float* x, float* y, int64_t n, float sg, float amp, int fast,
                                  int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(x) && aligned16(y)) ? n / 4 : 0;
  const LaunchShape ls = baseline_shape(n4, n, num_cu);
  const float c = (float)(-1.0 / (2.0 * (double)sg * (double)sg));
  if (fast)
    hipLaunchKernelGGL(k_direct_gaussian<true>, dim3(ls.grid), dim3(ls.block), 0, s, x, y, n4, n, c, amp);
  else
    hipLaunchKernelGGL(k_direct_gaussian<false>, dim3(ls.grid), dim3(ls.block), 0, s, x, y, n4, n, c, amp);
  return hipGetLastError();
}

hipError_t launch_direct_func(const FuncDesc& f, const float* x, float* y, int64_t n, int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(x) && aligned16(y)) ? n / 4 : 0;
  const LaunchShape ls = baseline_shape(n4, n, num_cu);
  hipLaunchKernelGGL(k_direct_func, dim3(ls.grid), dim3(ls.block), 0, s, f, x, y, n4, n);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, int64_t n, int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(src) && aligned16(dst)) ? n / 4 : 0;
  const int64_t per_wg = (int64_t)kCopyBlock * kCopyUnroll;
  const int64_t work = (n4 > 0) ? (n4 + per_wg - 1) / per_wg : (n + kCopyBlock - 1) / kCopyBlock;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * kCopyWgPerCu, work));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kCopyBlock), 0, s, src, dst, n4, n);
  return hipGetLastError();
}

}  // namespace pwl
