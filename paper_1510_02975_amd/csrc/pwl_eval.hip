// Streaming evaluation kernels (Algorithm 1, Sec. IV) for gfx950.
//
// Every workgroup stages the whole table in LDS once - packed records
// {x_k, v_k, slope_k, 1/h_k}, the interior knots (+inf padded) and the
// uniform index map - and then streams its share of the points with 16-byte
// non-temporal loads and stores, U vectors per thread in flight.  The path is
// a memory-bound gather (8 bytes per point forward, 16 fused forward and
// backward), so there is no matrix-core work: the only per-point work is the
// map lookup, a short knot compare loop in LDS, one 16-byte record read and
// one FMA.  The backward accumulates dL/dv in LDS with FP32 atomics and
// flushes it once per workgroup with global FP32 atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwl_internal.h"
#include "pwl_locate.h"

namespace pwl {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kUnroll = 4;         // float4 vectors per thread per iteration
constexpr int kMaxThreadsPerCU = 2048;
constexpr size_t kLdsPerCU = 160 * 1024;

struct Smem {
  float4* rec;
  float* knot;
  uint32_t* cell;
  float* dv;
};

__device__ __forceinline__ Smem carve(void* base, int N, int K, bool backward) {
  Smem s;
  s.rec = reinterpret_cast<float4*>(base);
  s.knot = reinterpret_cast<float*>(s.rec + N);
  s.cell = reinterpret_cast<uint32_t*>(s.knot + N + kKnotPad);
  s.dv = backward ? reinterpret_cast<float*>(s.cell + K) : nullptr;
  return s;
}

// Copy the table into LDS.  With v_override the vertex values come from the
// caller and slopes are re-derived as (v_{k+1} - v_k) / h_k in FP32.
__device__ __forceinline__ void stage_table(const EvalTable& t, const float* __restrict__ vo,
                                            const Smem& s) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = tid; k < t.N; k += nt) {
    float4 r = t.rec[k];
    if (vo != nullptr) {
      const float v0 = vo[k], v1 = vo[k + 1];
      r.y = v0;
      r.z = (v1 - v0) * r.w;
    }
    s.rec[k] = r;
  }
  const float inf = __builtin_inff();
  for (int k = tid; k < t.N + kKnotPad; k += nt)
    s.knot[k] = (k >= 1 && k <= t.N - 1) ? t.knots[k] : inf;
  for (int u = tid; u < t.K; u += nt) s.cell[u] = t.cells[u];
}

__device__ __forceinline__ float clamp_nan(float x, float a, float b) {
  return (x < a) ? a : ((x > b) ? b : x);   // NaN passes through
}

__device__ __forceinline__ float eval_point(float x, const EvalTable& t, const Smem& s) {
  const int seg = locate_segment(x, s.knot, s.cell, t.a32, t.scale32, t.K);
  const float4 r = s.rec[seg];
  return fmaf(clamp_nan(x, t.a32, t.b32) - r.x, r.z, r.y);
}

template <bool WY, bool WDX, bool WDV>
__device__ __forceinline__ void backward_point(float x, float g, const EvalTable& t, const Smem& s,
                                               float& y, float& dx) {
  const int seg = locate_segment(x, s.knot, s.cell, t.a32, t.scale32, t.K);
  const float4 r = s.rec[seg];
  const float d = clamp_nan(x, t.a32, t.b32) - r.x;
  if (WY) y = fmaf(d, r.z, r.y);
  if (WDX) {
    const bool inside = (x >= t.a32) && (x <= t.b32);
    dx = inside ? g * r.z : ((x != x) ? x : 0.0f);
  }
  if (WDV) {
    if (x == x) {
      const float w1 = (d * r.w) * g;   // delta g
      atomicAdd(s.dv + seg, g - w1);    // (1 - delta) g
      atomicAdd(s.dv + seg + 1, w1);
    }
  }
}

// Points [4 n4, n) (or all of them when the arrays are not 16-byte aligned,
// n4 = 0) go through this grid-strided scalar loop.
#define PWL_SCALAR_TAIL(...)                                                                \
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;         \
       i += (int64_t)gridDim.x * blockDim.x) {                                              \
    __VA_ARGS__;                                                                            \
  }

__global__ __launch_bounds__(1024) void k_eval_fwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ y, int64_t n4, int64_t n) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, false);
  stage_table(t, vo, s);
  __syncthreads();
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
        yv.x = eval_point(xv[u].x, t, s);
        yv.y = eval_point(xv[u].y, t, s);
        yv.z = eval_point(xv[u].z, t, s);
        yv.w = eval_point(xv[u].w, t, s);
        __builtin_nontemporal_store(yv, y4 + i);
      }
    }
  }
  PWL_SCALAR_TAIL(y[i] = eval_point(x[i], t, s))
}

template <bool WY, bool WDX, bool WDV>
__global__ __launch_bounds__(1024) void k_eval_bwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ y, float* __restrict__ dx,
                                                   float* __restrict__ dv, int64_t n4, int64_t n) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, WDV);
  stage_table(t, vo, s);
  if (WDV)
    for (int k = threadIdx.x; k <= t.N; k += blockDim.x) s.dv[k] = 0.0f;
  __syncthreads();
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x);
  const v4f* __restrict__ g4 = reinterpret_cast<const v4f*>(g);
  v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y);
  v4f* __restrict__ dx4 = reinterpret_cast<v4f*>(dx);
  const int64_t bs = blockDim.x;
  const int64_t stride = (int64_t)gridDim.x * bs * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * bs * kUnroll + threadIdx.x; base < n4; base += stride) {
    v4f xv[kUnroll], gv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) {
        xv[u] = __builtin_nontemporal_load(x4 + i);
        gv[u] = __builtin_nontemporal_load(g4 + i);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * bs;
      if (i < n4) {
        v4f yv, dxv;
        float yy = 0.0f, dd = 0.0f;
        backward_point<WY, WDX, WDV>(xv[u].x, gv[u].x, t, s, yy, dd); yv.x = yy; dxv.x = dd;
        backward_point<WY, WDX, WDV>(xv[u].y, gv[u].y, t, s, yy, dd); yv.y = yy; dxv.y = dd;
        backward_point<WY, WDX, WDV>(xv[u].z, gv[u].z, t, s, yy, dd); yv.z = yy; dxv.z = dd;
        backward_point<WY, WDX, WDV>(xv[u].w, gv[u].w, t, s, yy, dd); yv.w = yy; dxv.w = dd;
        if (WY) __builtin_nontemporal_store(yv, y4 + i);
        if (WDX) __builtin_nontemporal_store(dxv, dx4 + i);
      }
    }
  }
  PWL_SCALAR_TAIL({
    float yy = 0.0f, dd = 0.0f;
    backward_point<WY, WDX, WDV>(x[i], g[i], t, s, yy, dd);
    if (WY) y[i] = yy;
    if (WDX) dx[i] = dd;
  })
  if (WDV) {
    __syncthreads();
    for (int k = threadIdx.x; k <= t.N; k += blockDim.x) {
      const float v = s.dv[k];
      if (v != 0.0f) unsafeAtomicAdd(dv + k, v);
    }
  }
}

__global__ __launch_bounds__(1024) void k_locate(EvalTable t, const float* __restrict__ x,
                                                 int32_t* __restrict__ seg, int64_t n) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, false);
  stage_table(t, nullptr, s);
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    seg[i] = locate_segment(x[i], s.knot, s.cell, t.a32, t.scale32, t.K);
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

template <bool kFast>
__global__ __launch_bounds__(256) void k_direct_gaussian(const float* __restrict__ x,
                                                         float* __restrict__ y, int64_t n4, int64_t n,
                                                         float c, float amp) {
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

__global__ __launch_bounds__(256) void k_copy(const float* __restrict__ src, float* __restrict__ dst,
                                              int64_t n4, int64_t n) {
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

// Occupancy-driven launch shape: as many workgroups per CU as the table's LDS
// allows (at most 8), each big enough that a CU runs 2048 threads, and never
// more workgroups than there are vectors to process.
LaunchShape stream_shape(size_t lds, int64_t n4, int64_t n, int num_cu) {
  int wg_per_cu = (int)std::min<size_t>(8, std::max<size_t>(1, kLdsPerCU / std::max<size_t>(lds, 1)));
  int block = kMaxThreadsPerCU / wg_per_cu;
  block = std::max(256, std::min(1024, (block / 64) * 64));
  const int64_t work = (n4 > 0) ? (n4 + (int64_t)block * kUnroll - 1) / ((int64_t)block * kUnroll)
                                : (n + block - 1) / block;
  int64_t grid = (int64_t)num_cu * wg_per_cu;
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, work));
  return LaunchShape{block, (int)grid, lds};
}

}  // namespace

hipError_t launch_eval(const EvalTable& t, const float* vo, const float* x, float* y, int64_t n,
                       int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(x) && aligned16(y)) ? n / 4 : 0;
  const LaunchShape ls = stream_shape(eval_lds_bytes(t.N, t.K, false), n4, n, num_cu);
  hipLaunchKernelGGL(k_eval_fwd, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, x, y, n4, n);
  return hipGetLastError();
}

hipError_t launch_eval_backward(const EvalTable& t, const float* vo, const float* x, const float* g,
                                float* y, float* dx, float* dv, int64_t n, int num_cu, hipStream_t s) {
  const bool al = aligned16(x) && aligned16(g) && (y == nullptr || aligned16(y)) &&
                  (dx == nullptr || aligned16(dx));
  const int64_t n4 = al ? n / 4 : 0;
  const bool wdv = dv != nullptr;
  const LaunchShape ls = stream_shape(eval_lds_bytes(t.N, t.K, wdv), n4, n, num_cu);
  if (wdv) hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, s, dv, (int64_t)t.N + 1);
  const int key = (y != nullptr ? 4 : 0) | (dx != nullptr ? 2 : 0) | (wdv ? 1 : 0);
#define PWL_BWD_CASE(K, A, B, C)                                                              \
  case K:                                                                                     \
    hipLaunchKernelGGL((k_eval_bwd<A, B, C>), dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, \
                       x, g, y, dx, dv, n4, n);                                               \
    break;
  switch (key) {
    PWL_BWD_CASE(1, false, false, true)
    PWL_BWD_CASE(2, false, true, false)
    PWL_BWD_CASE(3, false, true, true)
    PWL_BWD_CASE(4, true, false, false)
    PWL_BWD_CASE(5, true, false, true)
    PWL_BWD_CASE(6, true, true, false)
    PWL_BWD_CASE(7, true, true, true)
    default:
      return hipErrorInvalidValue;
  }
#undef PWL_BWD_CASE
  return hipGetLastError();
}

hipError_t launch_locate(const EvalTable& t, const float* x, int32_t* seg, int64_t n, int num_cu,
                         hipStream_t s) {
  const LaunchShape ls = stream_shape(eval_lds_bytes(t.N, t.K, false), 0, n, num_cu);
  hipLaunchKernelGGL(k_locate, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, x, seg, n);
  return hipGetLastError();
}

hipError_t launch_direct_gaussian(const float* x, float* y, int64_t n, float sg, float amp, int fast,
                                  int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(x) && aligned16(y)) ? n / 4 : 0;
  const int block = 256;
  const int64_t work = (n4 > 0) ? (n4 + block * kUnroll - 1) / (block * kUnroll) : (n + block - 1) / block;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * 8, work));
  const float c = (float)(-1.0 / (2.0 * (double)sg * (double)sg));
  if (fast)
    hipLaunchKernelGGL(k_direct_gaussian<true>, dim3(grid), dim3(block), 0, s, x, y, n4, n, c, amp);
  else
    hipLaunchKernelGGL(k_direct_gaussian<false>, dim3(grid), dim3(block), 0, s, x, y, n4, n, c, amp);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, int64_t n, int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(src) && aligned16(dst)) ? n / 4 : 0;
  const int block = 256;
  const int64_t work = (n4 > 0) ? (n4 + block * kUnroll - 1) / (block * kUnroll) : (n + block - 1) / block;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * 8, work));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(block), 0, s, src, dst, n4, n);
  return hipGetLastError();
}

hipError_t configure_eval_kernels(int max_lds) {
  const int lim = max_lds < (int)kLdsPerCU ? max_lds : (int)kLdsPerCU;
  hipError_t e = hipFuncSetAttribute((const void*)k_eval_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_locate, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e != hipSuccess) return e;
#define PWL_ATTR(A, B, C)                                                                     \
  e = hipFuncSetAttribute((const void*)k_eval_bwd<A, B, C>,                                   \
                          hipFuncAttributeMaxDynamicSharedMemorySize, lim);                   \
  if (e != hipSuccess) return e;
  PWL_ATTR(false, false, true)
  PWL_ATTR(false, true, false)
  PWL_ATTR(false, true, true)
  PWL_ATTR(true, false, false)
  PWL_ATTR(true, false, true)
  PWL_ATTR(true, true, false)
  PWL_ATTR(true, true, true)
#undef PWL_ATTR
  return hipSuccess;
}

}  // namespace pwl
