// Streaming evaluation kernels (Algorithm 1, Sec. IV) for gfx950.
//
// Every workgroup stages the whole table in LDS once - packed records
// {x_k, v_k, slope_k, x_{k+1}}, the interior knots (NaN padded) and the
// uniform index map - and then streams its share of the points with 16-byte
// non-temporal loads and stores, U vectors per thread in flight.  The path is
// a memory-bound gather (8 bytes per point forward, 16 fused forward and
// backward), so there is no matrix-core work: the only per-point work is the
// map lookup, a short knot compare loop in LDS, one record read (12 of its
// 16 bytes; the backward reads all 16) and one FMA.  The backward
// accumulates dL/dv in LDS with FP64 atomics and writes one column of
// per-workgroup partial sums, which k_dv_reduce adds.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwl_internal.h"
#include "pwl_locate.h"
#include "pwl_stream.h"

namespace pwl {

namespace {

constexpr size_t kLdsPerCU = 160 * 1024;
constexpr int kXcds = 8;             // MI355X accelerator complex dies; workgroups go to them round-robin
constexpr int64_t kMinPointsPerWG = int64_t(1) << 15;   // streaming grids: points per workgroup, at least
constexpr int64_t kPointsPerStagedByte = 2;             // and per byte of table the workgroup stages

using namespace stream;

template <int U, class S>
__device__ __forceinline__ void eval_fwd_body(const EvalTable& t, const S& s, const float* __restrict__ x,
                                              float* __restrict__ y, int64_t n, int flags) {
  const int64_t blk = blockIdx.x, nblk = gridDim.x;
  const bool vec = (flags & 1) != 0;
  if (flags & 2) {   // PWL_LOCATE_SEARCH
    fwd_range<U, -1>(t, s, x, y, 0, n, vec, blk, nblk);
    return;
  }
  switch (t.meta[1]) {
    case 0:
    case 1: fwd_range<U, 1>(t, s, x, y, 0, n, vec, blk, nblk); break;
    case 2: fwd_range<U, 2>(t, s, x, y, 0, n, vec, blk, nblk); break;
    case 3: fwd_range<U, 3>(t, s, x, y, 0, n, vec, blk, nblk); break;
    case 4: fwd_range<U, 4>(t, s, x, y, 0, n, vec, blk, nblk); break;
    default: fwd_range<U, 0>(t, s, x, y, 0, n, vec, blk, nblk); break;
  }
}

// REC is the arrangement of the per-segment data in LDS (pwl_set_records):
// packed records, structure of arrays, or value/slope pairs.
template <int U, int REC>
__global__ __launch_bounds__(1024) void k_eval_fwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ y, int64_t n, int flags) {
  extern __shared__ float4 lds_f4[];
  if constexpr (REC == PWL_RECORDS_SOA) {
    const SmemSoA s = carve_soa(lds_f4, t.N, t.K);
    stage_table(t, vo, s);
    __syncthreads();
    eval_fwd_body<U>(t, s, x, y, n, flags);
  } else if constexpr (REC == PWL_RECORDS_PAIRS) {
    const SmemPairs s = carve_pairs(lds_f4, t.N, t.K);
    stage_table_pairs(t, vo, s);
    __syncthreads();
    eval_fwd_body<U>(t, s, x, y, n, flags);
  } else {
    const Smem s = carve(lds_f4, t.N, t.K, false);
    stage_table(t, vo, s);
    __syncthreads();
    eval_fwd_body<U>(t, s, x, y, n, flags);
  }
}

template <int U, bool WY, bool WDX, bool WDV>
__global__ __launch_bounds__(1024) void k_eval_bwd(EvalTable t, const float* __restrict__ vo,
                                                   const float* __restrict__ x,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ y, float* __restrict__ dx,
                                                   float* __restrict__ part, int64_t n, int vec) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, WDV);
  stage_table(t, vo, s);
  if (WDV)
    for (int k = threadIdx.x; k < (t.N + 1) * s.dvc; k += blockDim.x) s.dv[k] = 0.0;
  __syncthreads();
  using B = Bwd<U, WY, WDX, WDV>;
  const int64_t blk = blockIdx.x, nblk = gridDim.x;
  switch (t.meta[1]) {
    case 0:
    case 1: B::template range<1>(t, s, x, g, y, dx, 0, n, vec != 0, blk, nblk); break;
    case 2: B::template range<2>(t, s, x, g, y, dx, 0, n, vec != 0, blk, nblk); break;
    case 3: B::template range<3>(t, s, x, g, y, dx, 0, n, vec != 0, blk, nblk); break;
    case 4: B::template range<4>(t, s, x, g, y, dx, 0, n, vec != 0, blk, nblk); break;
    default: B::template range<0>(t, s, x, g, y, dx, 0, n, vec != 0, blk, nblk); break;
  }
  if (WDV) {
    // This workgroup's dL/dv becomes column `col` of the partial sums
    // part[k][col] (no atomics: k_dv_reduce adds each row in a fixed order).
    // Workgroups are dealt to the 8 XCDs round-robin, so the columns are
    // ordered XCD by XCD: the workgroups of one XCD fill whole cache lines
    // in their own L2.
    __syncthreads();
    const int G = gridDim.x, b = blockIdx.x;
    const int col = (G % kXcds == 0) ? (b % kXcds) * (G / kXcds) + b / kXcds : b;
    for (int k = threadIdx.x; k <= t.N; k += blockDim.x) {
      double acc = s.dv[k * s.dvc];
      for (int j = 1; j < s.dvc; ++j) acc += s.dv[k * s.dvc + j];   // the copies, in a fixed order
      part[(int64_t)k * G + col] = (float)acc;
    }
  }
}

// dL/dv[k] = the sum of row k of part[k][0..G), in FP64 and a fixed order:
// one wave per row, lane l adding columns l, l + 64, ... (coalesced 256-byte
// loads, all issued before the first add), then a butterfly over the lanes.
constexpr int kReduceThreads = 256;
__global__ __launch_bounds__(kReduceThreads) void k_dv_reduce(const float* __restrict__ part, int G, int N1,
                                                              float* __restrict__ dv) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (kReduceThreads / 64) + (threadIdx.x >> 6);
  if (k >= N1) return;   // whole waves leave together
  const float* row = part + (int64_t)k * G;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = lane;
  for (; c + 192 < G; c += 256) {
    s0 += (double)row[c];
    s1 += (double)row[c + 64];
    s2 += (double)row[c + 128];
    s3 += (double)row[c + 192];
  }
  for (; c < G; c += 64) s0 += (double)row[c];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) dv[k] = (float)s;
}

// Segment indices through the same locate the evaluation kernels run: the
// unrolled compare depth chosen from meta[1] (or the binary search), so the
// indices this returns are the ones k_eval_fwd, k_eval_bwd and the batched
// kernels use.
template <int MAXC>
__device__ __forceinline__ void locate_all(const EvalTable& t, const Smem& s, const float* __restrict__ x,
                                           int32_t* __restrict__ seg, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    seg[i] = locate<MAXC>(x[i], t, s);
}

__global__ __launch_bounds__(1024) void k_locate(EvalTable t, const float* __restrict__ x,
                                                 int32_t* __restrict__ seg, int64_t n, int flags) {
  extern __shared__ float4 lds_f4[];
  const Smem s = carve(lds_f4, t.N, t.K, false);
  stage_table(t, nullptr, s);
  __syncthreads();
  if (flags & 2) {   // PWL_LOCATE_SEARCH
    locate_all<-1>(t, s, x, seg, n);
    return;
  }
  switch (t.meta[1]) {
    case 0:
    case 1: locate_all<1>(t, s, x, seg, n); break;
    case 2: locate_all<2>(t, s, x, seg, n); break;
    case 3: locate_all<3>(t, s, x, seg, n); break;
    case 4: locate_all<4>(t, s, x, seg, n); break;
    default: locate_all<0>(t, s, x, seg, n); break;
  }
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// The vector path needs every point array at the same 16-byte phase (a
// slice of aligned arrays qualifies); the head and tail points are scalar.
inline bool same_phase(const void* a, const void* b) {
  return b == nullptr || ((reinterpret_cast<uintptr_t>(a) ^ reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
}

// Launch shape of a streaming evaluation kernel: workgroups of `block`
// threads, each thread handling `unroll` float4 vectors per iteration, on a
// grid of up to `wg_per_cu` workgroups per CU.  The grid may be many times
// what the CUs hold at once (register use caps residency at one 1024-thread
// workgroup per CU): workgroups are then dispatched as CUs free up, so CUs
// and XCDs that stream faster take more of the points, where a grid of one
// resident round waits for its slowest CU.  Each workgroup stages the whole
// table, so the grid is cut back, a whole workgroup per CU at a time (a
// partial last round leaves CUs idle), until a workgroup streams at least
// kMinPointsPerWG points and at least kPointsPerStagedByte points per byte
// of table it stages, but never below one workgroup per CU (nor above one
// per iteration of work).  The defaults are the autotuner's choice on
// MI355X: forward at 2^28 points, four vectors per thread in 1024-thread
// workgroups, up to 32 per CU (at N = 1024 the staging rule leaves 18,
// which measured 333 us against 335 us for 16; at N = 4096 it leaves about
// 3); fused backward at 2^26 points,
// two vectors per thread (the dL/dv LDS atomics favour a smaller register
// footprint) in one 768-thread workgroup per CU - every further workgroup
// there adds a dL/dv flush and a column to reduce.  The batched kernels
// take 1024-thread workgroups and four vectors per thread: the forward a
// persistent grid of 3 per CU, the fused backward 32 per CU (about one
// slice per workgroup, in rounds; its four-vector body spills a little and
// still measured 3% faster than two vectors in 3 per CU).  pwl_set_launch
// overrides them.
constexpr LaunchConfig kDefaultLaunch[4] = {{4, 1024, 32}, {2, 768, 1}, {4, 1024, 3}, {4, 1024, 32}};
LaunchConfig g_launch[4] = {kDefaultLaunch[0], kDefaultLaunch[1], kDefaultLaunch[2], kDefaultLaunch[3]};
int g_locate = PWL_LOCATE_MAP;
int g_records = PWL_RECORDS_PACKED;

LaunchShape stream_shape(const LaunchConfig& c, size_t lds, int64_t n4, int64_t n, int num_cu) {
  const int block = c.block;
  const int64_t per_wg = (int64_t)block * c.unroll;
  const int64_t work = (n4 > 0) ? (n4 + per_wg - 1) / per_wg : (n + block - 1) / block;
  const int64_t min_points = std::max<int64_t>(kMinPointsPerWG, kPointsPerStagedByte * (int64_t)lds);
  // whole workgroups per CU: a last partial round would leave CUs idle
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(c.wg_per_cu, n / (min_points * num_cu)));
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * per_cu, work));
  return LaunchShape{block, (int)grid, lds};
}

}  // namespace

hipError_t set_launch(int kernel, int unroll, int block, int wg_per_cu) {
  if (kernel < 0 || kernel > 3) return hipErrorInvalidValue;
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

hipError_t set_locate(int mode) {
  if (mode != PWL_LOCATE_MAP && mode != PWL_LOCATE_SEARCH) return hipErrorInvalidValue;
  g_locate = mode;
  return hipSuccess;
}

int get_locate() { return g_locate; }

hipError_t set_records(int layout) {
  if (layout != PWL_RECORDS_PACKED && layout != PWL_RECORDS_SOA && layout != PWL_RECORDS_PAIRS)
    return hipErrorInvalidValue;
  g_records = layout;
  return hipSuccess;
}

int get_records() { return g_records; }

hipError_t launch_eval(const EvalTable& t, const float* vo, const float* x, float* y, int64_t n,
                       int num_cu, hipStream_t s) {
  const bool vec = same_phase(x, y) && (reinterpret_cast<uintptr_t>(x) & 3u) == 0;
  const LaunchConfig c = g_launch[0];
  const int rec = g_records;
  const size_t lds = rec == PWL_RECORDS_SOA     ? eval_lds_bytes_soa(t.N, t.K)
                     : rec == PWL_RECORDS_PAIRS ? eval_lds_bytes_pairs(t.N, t.K)
                                                : eval_lds_bytes(t.N, t.K, false);
  const LaunchShape ls = stream_shape(c, lds, vec ? n / 4 : 0, n, num_cu);
  const int v = (vec ? 1 : 0) | (g_locate == PWL_LOCATE_SEARCH ? 2 : 0);
#define PWL_FWD(UU, RR) \
  hipLaunchKernelGGL((k_eval_fwd<UU, RR>), dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, x, y, n, v)
#define PWL_FWD_U(RR)                   \
  switch (c.unroll) {                   \
    case 1: PWL_FWD(1, RR); break;      \
    case 2: PWL_FWD(2, RR); break;      \
    default: PWL_FWD(4, RR); break;     \
  }
  if (rec == PWL_RECORDS_SOA) {
    PWL_FWD_U(PWL_RECORDS_SOA)
  } else if (rec == PWL_RECORDS_PAIRS) {
    PWL_FWD_U(PWL_RECORDS_PAIRS)
  } else {
    PWL_FWD_U(PWL_RECORDS_PACKED)
  }
#undef PWL_FWD_U
#undef PWL_FWD
  return hipGetLastError();
}

template <int U>
void launch_bwd_u(const LaunchShape& ls, int key, const EvalTable& t, const float* vo, const float* x,
                  const float* g, float* y, float* dx, float* part, int64_t n, int vec, hipStream_t s) {
#define PWL_BWD_CASE(K, A, B, C)                                                                 \
  case K:                                                                                        \
    hipLaunchKernelGGL((k_eval_bwd<U, A, B, C>), dim3(ls.grid), dim3(ls.block), ls.lds, s, t, vo, \
                       x, g, y, dx, part, n, vec);                                               \
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

LaunchShape backward_shape(const EvalTable& t, const float* x, const float* g, const float* y, const float* dx,
                           bool wdv, int64_t n, int num_cu) {
  const bool vec = same_phase(x, g) && same_phase(x, y) && same_phase(x, dx) &&
                   (reinterpret_cast<uintptr_t>(x) & 3u) == 0;
  return stream_shape(g_launch[1], eval_lds_bytes(t.N, t.K, wdv), vec ? n / 4 : 0, n, num_cu);
}

size_t backward_workspace_floats(const EvalTable& t, const float* x, const float* g, const float* y,
                                 const float* dx, int64_t n, int num_cu) {
  const LaunchShape ls = backward_shape(t, x, g, y, dx, true, n, num_cu);
  return (size_t)ls.grid * (size_t)(t.N + 1);
}

hipError_t launch_eval_backward(const EvalTable& t, const float* vo, const float* x, const float* g,
                                float* y, float* dx, float* dv, float* part, int64_t n, int num_cu,
                                hipStream_t s) {
  const bool vec = same_phase(x, g) && same_phase(x, y) && same_phase(x, dx) &&
                   (reinterpret_cast<uintptr_t>(x) & 3u) == 0;
  const bool wdv = dv != nullptr;
  const LaunchConfig c = g_launch[1];
  const LaunchShape ls = backward_shape(t, x, g, y, dx, wdv, n, num_cu);
  const int key = (y != nullptr ? 4 : 0) | (dx != nullptr ? 2 : 0) | (wdv ? 1 : 0);
  if (key == 0) return hipErrorInvalidValue;
  if (wdv && n == 0) {   // no points: dL/dv = 0
    hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, s, dv, (int64_t)t.N + 1);
    return hipGetLastError();
  }
  if (wdv && part == nullptr) return hipErrorInvalidValue;
  const int v = vec ? 1 : 0;
  switch (c.unroll) {
    case 1: launch_bwd_u<1>(ls, key, t, vo, x, g, y, dx, part, n, v, s); break;
    case 2: launch_bwd_u<2>(ls, key, t, vo, x, g, y, dx, part, n, v, s); break;
    default: launch_bwd_u<4>(ls, key, t, vo, x, g, y, dx, part, n, v, s); break;
  }
  if (wdv) {
    const int n1 = t.N + 1, rows_per_wg = kReduceThreads / 64;
    hipLaunchKernelGGL(k_dv_reduce, dim3((n1 + rows_per_wg - 1) / rows_per_wg), dim3(kReduceThreads), 0, s,
                       part, ls.grid, n1, dv);
  }
  return hipGetLastError();
}


hipError_t launch_locate(const EvalTable& t, const float* x, int32_t* seg, int64_t n, int num_cu,
                         hipStream_t s) {
  const LaunchShape ls = stream_shape(g_launch[0], eval_lds_bytes(t.N, t.K, false), 0, n, num_cu);
  const int v = (g_locate == PWL_LOCATE_SEARCH) ? 2 : 0;
  hipLaunchKernelGGL(k_locate, dim3(ls.grid), dim3(ls.block), ls.lds, s, t, x, seg, n, v);
  return hipGetLastError();
}

hipError_t configure_eval_kernels(int max_lds) {
  const int lim = max_lds < (int)kLdsPerCU ? max_lds : (int)kLdsPerCU;
  hipError_t e = hipSuccess;
#define PWL_ATTR(K)                                                                           \
  e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, lim);    \
  if (e != hipSuccess) return e;
  PWL_ATTR(k_locate)
#define PWL_ATTR_R(RR)                   \
  PWL_ATTR((k_eval_fwd<1, RR>))          \
  PWL_ATTR((k_eval_fwd<2, RR>))          \
  PWL_ATTR((k_eval_fwd<4, RR>))
  PWL_ATTR_R(PWL_RECORDS_PACKED)
  PWL_ATTR_R(PWL_RECORDS_SOA)
  PWL_ATTR_R(PWL_RECORDS_PAIRS)
#undef PWL_ATTR_R
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
