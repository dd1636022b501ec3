// Batched evaluation of many tables of uneven size over uneven point counts
// in one launch.
//
// The points of all tables are concatenated (table t owns [off_t, off_{t+1})).
// The host cuts them into one contiguous chunk of equal cost per workgroup
// (the grid holds many workgroups per CU, dispatched as CUs free up) and
// lists, per workgroup, the (table, begin, end) runs its chunk covers.  A
// workgroup walks its runs in order, re-staging the LDS table only when the
// table changes, and streams each run with the same vectorised body as the
// single-table evaluator.  The fused backward keeps a workgroup's dL/dv of
// the current table in FP64 LDS and flushes it with global FP32 atomics into
// the concatenated gradient (table t at dv_off_t) whenever the table changes
// and at the end.
#include <hip/hip_runtime.h>

#include "pwl_internal.h"
#include "pwl_stream.h"

namespace pwl {

namespace {

using namespace stream;

// The shape of a run's table as the streaming building blocks expect it (the
// array pointers are unused: the table is already in LDS).
__device__ __forceinline__ EvalTable run_table(const BatchRun& r) {
  EvalTable t;
  t.rec = nullptr;
  t.knots = nullptr;
  t.lo = nullptr;
  t.meta = nullptr;
  t.N = r.N;
  t.K = r.K;
  t.a32 = r.a32;
  t.b32 = r.b32;
  t.scale32 = r.scale32;
  return t;
}

// Linear copy of n 16-byte words (descriptors or a table image) into LDS.
__device__ __forceinline__ void copy_words(const float4* __restrict__ src, int n, float4* dst) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

template <int U>
__device__ __forceinline__ void batch_fwd_run(const BatchRun& r, const Smem& s, const float* __restrict__ x,
                                              float* __restrict__ y, bool vec) {
  const EvalTable t = run_table(r);
  switch (r.maxc) {
    case 0:
    case 1: fwd_run<U, 1>(t, s, x, y, r.begin, r.end, vec); break;
    case 2: fwd_run<U, 2>(t, s, x, y, r.begin, r.end, vec); break;
    case 3: fwd_run<U, 3>(t, s, x, y, r.begin, r.end, vec); break;
    case 4: fwd_run<U, 4>(t, s, x, y, r.begin, r.end, vec); break;
    default: fwd_run<U, 0>(t, s, x, y, r.begin, r.end, vec); break;
  }
}

// A workgroup walks its runs in blocks of kRunSlots descriptors held in LDS;
// it re-stages the table image only when the table changes.
template <int U>
__global__ __launch_bounds__(1024) void k_batch_fwd(const BatchRun* __restrict__ runs,
                                                    const int32_t* __restrict__ run_begin,
                                                    const float* __restrict__ x, float* __restrict__ y,
                                                    int vec) {
  extern __shared__ float4 lds_f4[];
  BatchRun* slots = reinterpret_cast<BatchRun*>(lds_f4);
  float4* image = lds_f4 + kRunSlots * (int)(sizeof(BatchRun) / 16);
  const int r0 = run_begin[blockIdx.x], r1 = run_begin[blockIdx.x + 1];
  int cur = -1;
  for (int rb = r0; rb < r1; rb += kRunSlots) {
    const int nr = min(kRunSlots, r1 - rb);
    __syncthreads();   // every thread is done with the previous descriptors and table
    copy_words(reinterpret_cast<const float4*>(runs + rb), nr * (int)(sizeof(BatchRun) / 16), lds_f4);
    __syncthreads();
    for (int q = 0; q < nr; ++q) {
      const BatchRun r = slots[q];
      if (r.table != cur) {
        if (cur >= 0) __syncthreads();
        copy_words(r.img, r.nvec, image);
        __syncthreads();
        cur = r.table;
      }
      batch_fwd_run<U>(r, carve(image, r.N, r.K, false), x, y, vec != 0);
    }
  }
}

template <int U, bool WY, bool WDX>
__device__ __forceinline__ void batch_bwd_run(const BatchRun& r, const Smem& s, const float* __restrict__ x,
                                              const float* __restrict__ g, float* __restrict__ y,
                                              float* __restrict__ dx, bool vec) {
  using B = Bwd<U, WY, WDX, true>;
  const EvalTable t = run_table(r);
  switch (r.maxc) {
    case 0:
    case 1: B::template range<1>(t, s, x, g, y, dx, r.begin, r.end, vec, 0, 1); break;
    case 2: B::template range<2>(t, s, x, g, y, dx, r.begin, r.end, vec, 0, 1); break;
    case 3: B::template range<3>(t, s, x, g, y, dx, r.begin, r.end, vec, 0, 1); break;
    case 4: B::template range<4>(t, s, x, g, y, dx, r.begin, r.end, vec, 0, 1); break;
    default: B::template range<0>(t, s, x, g, y, dx, r.begin, r.end, vec, 0, 1); break;
  }
}

__device__ __forceinline__ void flush_dv(const Smem& s, int N, float* __restrict__ dv) {
  for (int k = threadIdx.x; k <= N; k += blockDim.x) {
    const float v = (float)s.dv[k];
    if (v != 0.0f) unsafeAtomicAdd(dv + k, v);
  }
}

// As k_batch_fwd; the current table's dL/dv is kept in FP64 LDS and flushed
// with global FP32 atomics into the concatenated gradient whenever the table
// changes and at the end.
template <int U, bool WY, bool WDX>
__global__ __launch_bounds__(1024) void k_batch_bwd(const BatchRun* __restrict__ runs,
                                                    const int32_t* __restrict__ run_begin,
                                                    const float* __restrict__ x, const float* __restrict__ g,
                                                    float* __restrict__ y, float* __restrict__ dx,
                                                    float* __restrict__ dv, int vec) {
  extern __shared__ float4 lds_f4[];
  BatchRun* slots = reinterpret_cast<BatchRun*>(lds_f4);
  float4* image = lds_f4 + kRunSlots * (int)(sizeof(BatchRun) / 16);
  const int r0 = run_begin[blockIdx.x], r1 = run_begin[blockIdx.x + 1];
  int cur = -1, curN = 0;
  int64_t cur_off = 0;
  Smem s = carve(image, 0, 0, true);
  for (int rb = r0; rb < r1; rb += kRunSlots) {
    const int nr = min(kRunSlots, r1 - rb);
    __syncthreads();   // every thread is done with the previous descriptors
    copy_words(reinterpret_cast<const float4*>(runs + rb), nr * (int)(sizeof(BatchRun) / 16), lds_f4);
    __syncthreads();
    for (int q = 0; q < nr; ++q) {
      const BatchRun r = slots[q];
      if (r.table != cur) {
        if (cur >= 0) {
          __syncthreads();   // every thread is done with the previous table
          flush_dv(s, curN, dv + cur_off);
          __syncthreads();
        }
        copy_words(r.img, r.nvec, image);
        s = carve(image, r.N, r.K, true);
        for (int k = threadIdx.x; k <= r.N; k += blockDim.x) s.dv[k] = 0.0;
        __syncthreads();
        cur = r.table;
        curN = r.N;
        cur_off = r.dv_off;
      }
      batch_bwd_run<U, WY, WDX>(r, s, x, g, y, dx, vec != 0);
    }
  }
  if (cur >= 0) {
    __syncthreads();
    flush_dv(s, curN, dv + cur_off);
  }
}

// One workgroup per table: its LDS image (records, knots with NaN outside
// 1..N-1 up to the sentinel pad, index map, zero padding to whole 16-byte
// words) and its deepest map cell.
__global__ __launch_bounds__(256) void k_batch_pack(const BatchTable* __restrict__ tabs, int32_t* __restrict__ maxc) {
  const BatchTable bt = tabs[blockIdx.x];
  const EvalTable& t = bt.t;
  stage_table(t, nullptr, carve(bt.img, t.N, t.K, false));   // the same words a kernel stages
  if (threadIdx.x == 0) maxc[blockIdx.x] = (int32_t)t.meta[1];
}

__global__ void k_batch_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

inline bool same_phase(const void* a, const void* b) {
  return b == nullptr || ((reinterpret_cast<uintptr_t>(a) ^ reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
}

hipError_t launch_plan(const BatchLaunch& bl, const BatchPlan& p, const LaunchConfig& c, const float* x,
                       const float* g, float* y, float* dx, float* dv, int v, hipStream_t s) {
  const dim3 grid(p.grid), block(c.block);
  if (g == nullptr) {
    switch (c.unroll) {
      case 1: hipLaunchKernelGGL(k_batch_fwd<1>, grid, block, p.lds, s, p.runs, p.run_begin, x, y, v); break;
      case 2: hipLaunchKernelGGL(k_batch_fwd<2>, grid, block, p.lds, s, p.runs, p.run_begin, x, y, v); break;
      default: hipLaunchKernelGGL(k_batch_fwd<4>, grid, block, p.lds, s, p.runs, p.run_begin, x, y, v); break;
    }
    return hipGetLastError();
  }
  const int key = (y != nullptr ? 2 : 0) | (dx != nullptr ? 1 : 0);
#define PWL_BB(UU, A, B)                                                                              \
  hipLaunchKernelGGL((k_batch_bwd<UU, A, B>), grid, block, p.lds, s, p.runs, p.run_begin, x, g, \
                     y, dx, dv, v)
#define PWL_BB_U(UU)                             \
  switch (key) {                                 \
    case 0: PWL_BB(UU, false, false); break;     \
    case 1: PWL_BB(UU, false, true); break;      \
    case 2: PWL_BB(UU, true, false); break;      \
    default: PWL_BB(UU, true, true); break;      \
  }
  switch (c.unroll) {
    case 1: PWL_BB_U(1) break;
    case 2: PWL_BB_U(2) break;
    default: PWL_BB_U(4) break;
  }
#undef PWL_BB_U
#undef PWL_BB
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchLaunch& bl, const float* x, const float* g, float* y, float* dx,
                        float* dv, hipStream_t s) {
  const bool backward = g != nullptr;
  const LaunchConfig c = get_launch(backward ? PWL_KERNEL_BATCH_BACKWARD : PWL_KERNEL_BATCH);
  const bool vec = same_phase(x, y) && same_phase(x, g) && same_phase(x, dx) &&
                   (reinterpret_cast<uintptr_t>(x) & 3u) == 0;
  const int v = vec ? 1 : 0;
  if (backward) {
    const int64_t zgrid = std::min<int64_t>(1024, (bl.dv_len + 255) / 256);
    hipLaunchKernelGGL(k_batch_zero, dim3((unsigned)std::max<int64_t>(1, zgrid)), dim3(256), 0, s, dv, bl.dv_len);
  }
  const hipError_t e = launch_plan(bl, backward ? bl.bwd : bl.fwd, c, x, g, y, dx, dv, v, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_batch_pack(const BatchTable* tabs, int T, int32_t* maxc, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_pack, dim3(T), dim3(256), 0, s, tabs, maxc);
  return hipGetLastError();
}

hipError_t configure_batch_kernels(int max_lds) {
  const int lim = max_lds < 160 * 1024 ? max_lds : 160 * 1024;
  hipError_t e = hipSuccess;
#define PWL_ATTR(K)                                                                        \
  e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, lim); \
  if (e != hipSuccess) return e;
  PWL_ATTR(k_batch_fwd<1>)
  PWL_ATTR(k_batch_fwd<2>)
  PWL_ATTR(k_batch_fwd<4>)
#define PWL_ATTR_U(UU)                          \
  PWL_ATTR((k_batch_bwd<UU, false, false>))     \
  PWL_ATTR((k_batch_bwd<UU, false, true>))      \
  PWL_ATTR((k_batch_bwd<UU, true, false>))      \
  PWL_ATTR((k_batch_bwd<UU, true, true>))
  PWL_ATTR_U(1)
  PWL_ATTR_U(2)
  PWL_ATTR_U(4)
#undef PWL_ATTR_U
#undef PWL_ATTR
  return hipSuccess;
}

}  // namespace pwl
