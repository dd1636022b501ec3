// Batched evaluation of many tables of uneven size over uneven point counts
// in one launch.
//
// The points of all tables are concatenated (table t owns [off_t, off_{t+1})).
// The host cuts them into one contiguous chunk of equal cost per workgroup
// (the grid holds many workgroups per CU, dispatched as CUs free up) and
// lists, per workgroup, the (table, begin, end) runs its chunk covers.  A
// workgroup copies the LDS images of all its runs' tables - one contiguous
// span of the batch's image arena, the host having split chunks whose span
// would not fit - into LDS with one barrier, then streams its runs one after
// the other with the same vectorised body as the single-table evaluator and
// no barrier between them: a wave that finishes a run goes straight on to
// the next.  The fused backward keeps a dL/dv region in FP64 LDS per table
// of the workgroup and, after one more barrier, flushes each with global
// FP32 atomics into the concatenated gradient (table t at dv_off_t).
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

// Copies n >= 1 16-byte words from global memory to LDS, four per thread
// per round: each round issues all its loads before its first store.  The
// loads are unconditional (indices clamped to the last word): a load under
// a per-thread condition would make the compiler wait for it before the next.
__device__ __forceinline__ void stage_words(const float4* __restrict__ src4, int n, float4* dst4) {
  const v4f* __restrict__ src = reinterpret_cast<const v4f*>(src4);
  v4f* dst = reinterpret_cast<v4f*>(dst4);
  const int tid = threadIdx.x, bs = blockDim.x;
  for (int k0 = 0; k0 < n; k0 += 4 * bs) {
    v4f w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = src[min(k0 + j * bs + tid, n - 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j * bs + tid;
      if (k < n) dst[k] = w[j];
    }
  }
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

// One workgroup: stage the images of all its runs' tables, one barrier,
// then its runs one after the other.  The run descriptors are read from
// global memory (uniform: the scalar cache).
template <int U>
__global__ __launch_bounds__(1024) void k_batch_fwd(const BatchRun* __restrict__ runs,
                                                    const BatchGroup* __restrict__ groups,
                                                    const float4* __restrict__ arena,
                                                    const float* __restrict__ x, float* __restrict__ y,
                                                    int vec) {
  extern __shared__ float4 lds_f4[];
  const BatchGroup gp = groups[blockIdx.x];
  if (gp.r0 >= gp.r1) return;
  stage_words(arena + gp.img, gp.nwords, lds_f4);
  __syncthreads();
  for (int q = gp.r0; q < gp.r1; ++q) {
    const BatchRun r = runs[q];
    batch_fwd_run<U>(r, carve(lds_f4 + r.img_lds, r.N, r.K, false), x, y, vec != 0);
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

// As k_batch_fwd, with one FP64 dL/dv region per run's table after the
// images (zeroed before the barrier); after the runs, one more barrier and
// every region is flushed with global FP32 atomics.
template <int U, bool WY, bool WDX>
__global__ __launch_bounds__(1024) void k_batch_bwd(const BatchRun* __restrict__ runs,
                                                    const BatchGroup* __restrict__ groups,
                                                    const float4* __restrict__ arena,
                                                    const float* __restrict__ x, const float* __restrict__ g,
                                                    float* __restrict__ y, float* __restrict__ dx,
                                                    float* __restrict__ dv, int vec) {
  extern __shared__ float4 lds_f4[];
  const BatchGroup gp = groups[blockIdx.x];
  if (gp.r0 >= gp.r1) return;
  stage_words(arena + gp.img, gp.nwords, lds_f4);
  double* dvz = reinterpret_cast<double*>(lds_f4 + gp.dv_lds);
  for (int k = threadIdx.x; k < 2 * gp.dv_words; k += blockDim.x) dvz[k] = 0.0;
  __syncthreads();
  for (int q = gp.r0; q < gp.r1; ++q) {
    const BatchRun r = runs[q];
    Smem s = carve(lds_f4 + r.img_lds, r.N, r.K, false);
    s.dv = reinterpret_cast<double*>(lds_f4 + r.dv_lds);
    batch_bwd_run<U, WY, WDX>(r, s, x, g, y, dx, vec != 0);
  }
  __syncthreads();
  for (int q = gp.r0; q < gp.r1; ++q) {
    const BatchRun r = runs[q];
    const double* d = reinterpret_cast<const double*>(lds_f4 + r.dv_lds);
    float* out = dv + r.dv_off;
    for (int k = threadIdx.x; k <= r.N; k += blockDim.x) {
      const float v = (float)d[k];
      if (v != 0.0f) unsafeAtomicAdd(out + k, v);
    }
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
      case 1: hipLaunchKernelGGL(k_batch_fwd<1>, grid, block, p.lds, s, p.runs, p.groups, p.arena, x, y, v); break;
      case 2: hipLaunchKernelGGL(k_batch_fwd<2>, grid, block, p.lds, s, p.runs, p.groups, p.arena, x, y, v); break;
      default: hipLaunchKernelGGL(k_batch_fwd<4>, grid, block, p.lds, s, p.runs, p.groups, p.arena, x, y, v); break;
    }
    return hipGetLastError();
  }
  const int key = (y != nullptr ? 2 : 0) | (dx != nullptr ? 1 : 0);
#define PWL_BB(UU, A, B)                                                                              \
  hipLaunchKernelGGL((k_batch_bwd<UU, A, B>), grid, block, p.lds, s, p.runs, p.groups, p.arena, x, g, \
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
