// Streaming evaluation kernels (Algorithm 1, Sec. IV) for gfx950.
//
// Every workgroup stages the whole table in LDS once - packed records
// {x_k, v_k, slope_k, 1/h_k}, the interior knots (+inf padded) and the
// uniform index map - and then streams its share of the points with 16-byte
// non-temporal loads and stores, U vectors per thread in flight.  The path is
// a memory-bound gather (8 bytes per point forward, 16 fused forward and
// backward), so there is no matrix-core work: the only per-point work is the
// map lookup, a short knot compare loop in LDS, one 16-byte record read and
// one FMA.  The backward accumulates dL/dv in LDS with FP64 atomics and
// flushes it once per workgroup with global FP32 atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwl_internal.h"
#include "pwl_locate.h"

namespace pwl {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kStreamUnroll = 4;    // float4 vectors per thread per iteration (baselines)
constexpr size_t kLdsPerCU = 160 * 1024;

struct Smem {
  float4* rec;      // [N]           {x_k, v_k, slope_k, 1/h_k}
  float* knot;      // [N + pad]     knot[k] = x_k for 1 <= k <= N-1, NaN elsewhere
  uint16_t* lo;     // [K + 1]       lo[u] = #{interior knots in cells < u}; lo[K] = N - 1
  double* dv;       // [N + 1]       backward only: this workgroup's dL/dv
};

__device__ __forceinline__ Smem carve(void* base, int N, int K, bool backward) {
  Smem s;
  s.rec = reinterpret_cast<float4*>(base);
  s.knot = reinterpret_cast<float*>(s.rec + N);
  s.lo = reinterpret_cast<uint16_t*>(s.knot + N + kKnotPad);
  s.dv = backward ? reinterpret_cast<double*>(
                        (reinterpret_cast<uintptr_t>(s.lo + ((K + 2) & ~1)) + 7) & ~(uintptr_t)7)
                  : nullptr;
  return s;
}

// Copy the table into LDS.  With v_override the vertex values come from the
// caller and slopes are re-derived as (v_{k+1} - v_k) / h_k in FP32.  The
// knot sentinels are NaN so that every compare against them is false, even
// for x = +inf.
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
  const float qnan = __builtin_nanf("");
  for (int k = tid; k < t.N + kKnotPad; k += nt)
    s.knot[k] = (k >= 1 && k <= t.N - 1) ? t.knots[k] : qnan;
  for (int u = tid; u <= t.K; u += nt) s.lo[u] = t.lo[u];
}

__device__ __forceinline__ float clamp_nan(float x, float a, float b) {
  return (x < a) ? a : ((x > b) ? b : x);   // NaN passes through
}

// Segment of x when no map cell holds more than MAXC knots: compare x with
// the MAXC knots that follow lo[cell(x)].  Knots beyond the cell's own are
// greater than x (they lie in later cells) and the sentinels are NaN, so the
// extra compares are false; the count of true compares is exact.
template <int MAXC>
__device__ __forceinline__ int locate_fixed(float x, const EvalTable& t, const Smem& s) {
  const int u = map_cell(x, t.a32, t.scale32, t.K);
  const int lo = s.lo[u];
  int seg = lo;
#pragma unroll
  for (int j = 1; j <= MAXC; ++j) seg += (x >= s.knot[lo + j]) ? 1 : 0;
  return seg;
}

// Any number of knots per cell: the count is lo[u+1] - lo[u].
__device__ __forceinline__ int locate_any(float x, const EvalTable& t, const Smem& s) {
  const int u = map_cell(x, t.a32, t.scale32, t.K);
  const int lo = s.lo[u];
  const int cnt = (int)s.lo[u + 1] - lo;
  int seg = lo;
  for (int j = 1; j <= cnt; ++j) seg += (x >= s.knot[lo + j]) ? 1 : 0;
  return seg;
}

template <int MAXC>
__device__ __forceinline__ int locate(float x, const EvalTable& t, const Smem& s) {
  if (MAXC > 0) return locate_fixed<MAXC>(x, t, s);
  return locate_any(x, t, s);
}

template <int MAXC>
__device__ __forceinline__ float eval_point(float x, const EvalTable& t, const Smem& s) {
  const int seg = locate<MAXC>(x, t, s);
  const float4 r = s.rec[seg];
  return fmaf(clamp_nan(x, t.a32, t.b32) - r.x, r.z, r.y);
}

template <int MAXC, bool WY, bool WDX, bool WDV>
__device__ __forceinline__ void backward_point(float x, float g, const EvalTable& t, const Smem& s,
                                               float& y, float& dx) {
  const int seg = locate<MAXC>(x, t, s);
  const float4 r = s.rec[seg];
  const float d = clamp_nan(x, t.a32, t.b32) - r.x;
  if (WY) y = fmaf(d, r.z, r.y);
  if (WDX) {
    const bool inside = (x >= t.a32) && (x <= t.b32);
    dx = inside ? g * r.z : ((x != x) ? x : 0.0f);
  }
  if (WDV) {
    if (x == x) {
      // The workgroup's dL/dv lives in LDS as FP64: FP64 LDS atomic adds run
      // at full rate on gfx950 (FP32 ones take a slow path) and keep the
      // per-workgroup sums exact to FP32 output precision.  Workgroup scope,
      // relaxed: no point has to wait for the thread's outstanding stores.
      const float w1 = (d * r.w) * g;   // delta g
      __hip_atomic_fetch_add(s.dv + seg, (double)(g - w1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(s.dv + seg + 1, (double)w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

// One grid-stride iteration over U float4 vectors per thread: all loads,
// then all table lookups, then all stores.  Full iterations run unguarded so
// the compiler can count outstanding memory operations exactly (a guarded
// load makes every later wait a wait for all stores); the last, partial
// iteration of a thread is guarded.
template <int U, int MAXC, bool GUARD>
__device__ __forceinline__ void fwd_iter(const EvalTable& t, const Smem& s, const v4f* __restrict__ x4,
                                         v4f* __restrict__ y4, int64_t base, int64_t bs, int64_t n4) {
  v4f xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + u * bs;
    if (!GUARD || i < n4) xv[u] = __builtin_nontemporal_load(x4 + i);
  }
  v4f yv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    yv[u].x = eval_point<MAXC>(xv[u].x, t, s);
    yv[u].y = eval_point<MAXC>(xv[u].y, t, s);
    yv[u].z = eval_point<MAXC>(xv[u].z, t, s);
    yv[u].w = eval_point<MAXC>(xv[u].w, t, s);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + u * bs;
    if (!GUARD || i < n4) __builtin_nontemporal_store(yv[u], y4 + i);
  }
}

template <int U, int MAXC>
__device__ __forceinline__ void fwd_stream(const EvalTable& t, const Smem& s, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t n4, int64_t n) {
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x);
  v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y);
  const int64_t bs = blockDim.x;
  const int64_t stride = (int64_t)gridDim.x * bs * U;
  int64_t base = (int64_t)blockIdx.x * bs * U + threadIdx.x;
  for (; base + (U - 1) * bs < n4; base += stride) fwd_iter<U, MAXC, false>(t, s, x4, y4, base, bs, n4);
  if (base < n4) fwd_iter<U, MAXC, true>(t, s, x4, y4, base, bs, n4);
  PWL_SCALAR_TAIL(y[i] = eval_point<MAXC>(x[i], t, s))
}

template <int U>
__global__ __launch_bounds__(1024) void k_eval_fwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ y, int64_t n4, int64_t n) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, false);
  stage_table(t, vo, s);
  __syncthreads();
  switch (t.meta[1]) {
    case 0:
    case 1: fwd_stream<U, 1>(t, s, x, y, n4, n); break;
    case 2: fwd_stream<U, 2>(t, s, x, y, n4, n); break;
    case 3: fwd_stream<U, 3>(t, s, x, y, n4, n); break;
    case 4: fwd_stream<U, 4>(t, s, x, y, n4, n); break;
    default: fwd_stream<U, 0>(t, s, x, y, n4, n); break;
  }
}

template <int U, bool WY, bool WDX, bool WDV>
struct Bwd {
  template <int MAXC, bool GUARD>
  __device__ __forceinline__ static void iter(const EvalTable& t, const Smem& s, const v4f* __restrict__ x4,
                                              const v4f* __restrict__ g4, v4f* __restrict__ y4,
                                              v4f* __restrict__ dx4, int64_t base, int64_t bs, int64_t n4) {
    v4f xv[U], gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * bs;
      if (!GUARD || i < n4) {
        xv[u] = __builtin_nontemporal_load(x4 + i);
        gv[u] = __builtin_nontemporal_load(g4 + i);
      }
    }
    v4f yv[U], dxv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (GUARD && base + u * bs >= n4) continue;
      float yy = 0.0f, dd = 0.0f;
      backward_point<MAXC, WY, WDX, WDV>(xv[u].x, gv[u].x, t, s, yy, dd); yv[u].x = yy; dxv[u].x = dd;
      backward_point<MAXC, WY, WDX, WDV>(xv[u].y, gv[u].y, t, s, yy, dd); yv[u].y = yy; dxv[u].y = dd;
      backward_point<MAXC, WY, WDX, WDV>(xv[u].z, gv[u].z, t, s, yy, dd); yv[u].z = yy; dxv[u].z = dd;
      backward_point<MAXC, WY, WDX, WDV>(xv[u].w, gv[u].w, t, s, yy, dd); yv[u].w = yy; dxv[u].w = dd;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * bs;
      if (!GUARD || i < n4) {
        if (WY) __builtin_nontemporal_store(yv[u], y4 + i);
        if (WDX) __builtin_nontemporal_store(dxv[u], dx4 + i);
      }
    }
  }

  template <int MAXC>
  __device__ __forceinline__ static void stream(const EvalTable& t, const Smem& s,
                                                const float* __restrict__ x, const float* __restrict__ g,
                                                float* __restrict__ y, float* __restrict__ dx, int64_t n4,
                                                int64_t n) {
    const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x);
    const v4f* __restrict__ g4 = reinterpret_cast<const v4f*>(g);
    v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y);
    v4f* __restrict__ dx4 = reinterpret_cast<v4f*>(dx);
    const int64_t bs = blockDim.x;
    const int64_t stride = (int64_t)gridDim.x * bs * U;
    int64_t base = (int64_t)blockIdx.x * bs * U + threadIdx.x;
    for (; base + (U - 1) * bs < n4; base += stride)
      iter<MAXC, false>(t, s, x4, g4, y4, dx4, base, bs, n4);
    if (base < n4) iter<MAXC, true>(t, s, x4, g4, y4, dx4, base, bs, n4);
    PWL_SCALAR_TAIL({
      float yy = 0.0f, dd = 0.0f;
      backward_point<MAXC, WY, WDX, WDV>(x[i], g[i], t, s, yy, dd);
      if (WY) y[i] = yy;
      if (WDX) dx[i] = dd;
    })
  }
};

template <int U, bool WY, bool WDX, bool WDV>
__global__ __launch_bounds__(1024) void k_eval_bwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ y, float* __restrict__ dx,
                                                   float* __restrict__ dv, int64_t n4, int64_t n) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, WDV);
  stage_table(t, vo, s);
  if (WDV)
    for (int k = threadIdx.x; k <= t.N; k += blockDim.x) s.dv[k] = 0.0;
  __syncthreads();
  using B = Bwd<U, WY, WDX, WDV>;
  switch (t.meta[1]) {
    case 0:
    case 1: B::template stream<1>(t, s, x, g, y, dx, n4, n); break;
    case 2: B::template stream<2>(t, s, x, g, y, dx, n4, n); break;
    case 3: B::template stream<3>(t, s, x, g, y, dx, n4, n); break;
    case 4: B::template stream<4>(t, s, x, g, y, dx, n4, n); break;
    default: B::template stream<0>(t, s, x, g, y, dx, n4, n); break;
  }
  if (WDV) {
    __syncthreads();
    for (int k = threadIdx.x; k <= t.N; k += blockDim.x) {
      const float v = (float)s.dv[k];
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
    seg[i] = locate_any(x[i], t, s);
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

__global__ __launch_bounds__(256) void k_copy(const float* __restrict__ src, float* __restrict__ dst,
                                              int64_t n4, int64_t n) {
  constexpr int kUnroll = kStreamUnroll;
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

// Launch shape of a streaming evaluation kernel: `wg_per_cu` workgroups of
// `block` threads per CU (fewer if the table's LDS does not allow that
// many), each thread handling `unroll` float4 vectors per iteration, and
// never more workgroups than there are vectors.  The defaults are the
// autotuner's choice on MI355X for 2^28 points (forward and fused backward:
// four vectors per thread, two 1024-thread workgroups per CU); a shape with
// only a few resident workgroups per CU streams fastest.  pwl_set_launch
// overrides them.
constexpr LaunchConfig kDefaultLaunch[3] = {{4, 1024, 2}, {4, 1024, 2}, {4, 1024, 2}};
LaunchConfig g_launch[3] = {kDefaultLaunch[0], kDefaultLaunch[1], kDefaultLaunch[2]};

LaunchShape stream_shape(const LaunchConfig& c, size_t lds, int64_t n4, int64_t n, int num_cu) {
  const int wg_lds = (int)std::max<size_t>(1, kLdsPerCU / std::max<size_t>(lds, 1));
  const int wg_per_cu = std::max(1, std::min(c.wg_per_cu, wg_lds));
  const int block = c.block;
  const int64_t per_wg = (int64_t)block * c.unroll;
  const int64_t work = (n4 > 0) ? (n4 + per_wg - 1) / per_wg : (n + block - 1) / block;
  int64_t grid = (int64_t)num_cu * wg_per_cu;
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, work));
  return LaunchShape{block, (int)grid, lds};
}

}  // namespace

hipError_t set_launch(int kernel, int unroll, int block, int wg_per_cu) {
  if (kernel < 0 || kernel > 2) return hipErrorInvalidValue;
  if (unroll == 0 && block == 0 && wg_per_cu == 0) {
    g_launch[kernel] = kDefaultLaunch[kernel];
    return hipSuccess;
  }
  if (!(unroll == 1 || unroll == 2 || unroll == 4)) return hipErrorInvalidValue;
  if (block < 64 || block > 1024 || (block % 64) != 0) return hipErrorInvalidValue;
  if (wg_per_cu < 1 || wg_per_cu > 32) return hipErrorInvalidValue;
  g_launch[kernel] = LaunchConfig{unroll, block, wg_per_cu};
  return hipSuccess;
}

LaunchConfig get_launch(int kernel) { return g_launch[kernel]; }

hipError_t launch_eval(const EvalTable& t, const float* vo, const float* x, float* y, int64_t n,
                       int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(x) && aligned16(y)) ? n / 4 : 0;
  const LaunchConfig c = g_launch[0];
  const LaunchShape ls = stream_shape(c, eval_lds_bytes(t.N, t.K, false), n4, n, num_cu);
  switch (c.unroll) {
    case 1: hipLaunchKernelGGL(k_eval_fwd<1>, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, x, y, n4, n); break;
    case 2: hipLaunchKernelGGL(k_eval_fwd<2>, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, x, y, n4, n); break;
    default: hipLaunchKernelGGL(k_eval_fwd<4>, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, x, y, n4, n); break;
  }
  return hipGetLastError();
}

template <int U>
void launch_bwd_u(const LaunchShape& ls, int key, const EvalTable& t, const float* vo, const float* x,
                  const float* g, float* y, float* dx, float* dv, int64_t n4, int64_t n, hipStream_t s) {
#define PWL_BWD_CASE(K, A, B, C)                                                                 \
  case K:                                                                                        \
    hipLaunchKernelGGL((k_eval_bwd<U, A, B, C>), dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, \
                       x, g, y, dx, dv, n4, n);                                                  \
    break;
  switch (key) {
    PWL_BWD_CASE(1, false, false, true)
    PWL_BWD_CASE(2, false, true, false)
    PWL_BWD_CASE(3, false, true, true)
    PWL_BWD_CASE(4, true, false, false)
    PWL_BWD_CASE(5, true, false, true)
    PWL_BWD_CASE(6, true, true, false)
    PWL_BWD_CASE(7, true, true, true)
    default: break;
  }
#undef PWL_BWD_CASE
}

hipError_t launch_eval_backward(const EvalTable& t, const float* vo, const float* x, const float* g,
                                float* y, float* dx, float* dv, int64_t n, int num_cu, hipStream_t s) {
  const bool al = aligned16(x) && aligned16(g) && (y == nullptr || aligned16(y)) &&
                  (dx == nullptr || aligned16(dx));
  const int64_t n4 = al ? n / 4 : 0;
  const bool wdv = dv != nullptr;
  const LaunchConfig c = g_launch[1];
  const LaunchShape ls = stream_shape(c, eval_lds_bytes(t.N, t.K, wdv), n4, n, num_cu);
  const int key = (y != nullptr ? 4 : 0) | (dx != nullptr ? 2 : 0) | (wdv ? 1 : 0);
  if (key == 0) return hipErrorInvalidValue;
  if (wdv) hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, s, dv, (int64_t)t.N + 1);
  switch (c.unroll) {
    case 1: launch_bwd_u<1>(ls, key, t, vo, x, g, y, dx, dv, n4, n, s); break;
    case 2: launch_bwd_u<2>(ls, key, t, vo, x, g, y, dx, dv, n4, n, s); break;
    default: launch_bwd_u<4>(ls, key, t, vo, x, g, y, dx, dv, n4, n, s); break;
  }
  return hipGetLastError();
}

namespace {

LaunchShape baseline_shape(int64_t n4, int64_t n, int num_cu) {
  const int block = 256;
  const int64_t work = (n4 > 0) ? (n4 + block * kStreamUnroll - 1) / (block * kStreamUnroll)
                                : (n + block - 1) / block;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * 8, work));
  return LaunchShape{block, grid, 0};
}

}  // namespace

hipError_t launch_locate(const EvalTable& t, const float* x, int32_t* seg, int64_t n, int num_cu,
                         hipStream_t s) {
  const LaunchShape ls = stream_shape(g_launch[0], eval_lds_bytes(t.N, t.K, false), 0, n, num_cu);
  hipLaunchKernelGGL(k_locate, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, x, seg, n);
  return hipGetLastError();
}

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

hipError_t launch_copy(const float* src, float* dst, int64_t n, int num_cu, hipStream_t s) {
  const int64_t n4 = (aligned16(src) && aligned16(dst)) ? n / 4 : 0;
  const LaunchShape ls = baseline_shape(n4, n, num_cu);
  hipLaunchKernelGGL(k_copy, dim3(ls.grid), dim3(ls.block), 0, s, src, dst, n4, n);
  return hipGetLastError();
}

hipError_t configure_eval_kernels(int max_lds) {
  const int lim = max_lds < (int)kLdsPerCU ? max_lds : (int)kLdsPerCU;
  hipError_t e = hipSuccess;
#define PWL_ATTR(K)                                                                           \
  e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, lim);    \
  if (e != hipSuccess) return e;
  PWL_ATTR(k_locate)
  PWL_ATTR(k_eval_fwd<1>)
  PWL_ATTR(k_eval_fwd<2>)
  PWL_ATTR(k_eval_fwd<4>)
#define PWL_ATTR_U(U)                            \
  PWL_ATTR((k_eval_bwd<U, false, false, true>))  \
  PWL_ATTR((k_eval_bwd<U, false, true, false>))  \
  PWL_ATTR((k_eval_bwd<U, false, true, true>))   \
  PWL_ATTR((k_eval_bwd<U, true, false, false>))  \
  PWL_ATTR((k_eval_bwd<U, true, false, true>))   \
  PWL_ATTR((k_eval_bwd<U, true, true, false>))   \
  PWL_ATTR((k_eval_bwd<U, true, true, true>))
  PWL_ATTR_U(1)
  PWL_ATTR_U(2)
  PWL_ATTR_U(4)
#undef PWL_ATTR_U
#undef PWL_ATTR
  return hipSuccess;
}

}  // namespace pwl
