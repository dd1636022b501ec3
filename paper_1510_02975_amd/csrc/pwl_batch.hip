// Batched evaluation of many tables of uneven size over uneven point counts
// in one launch.
//
// The points of all tables are concatenated (table t owns [off_t, off_{t+1})).
//
// Forward: the host cuts the points into slices of a whole number of the
// kernel's vector iterations (two by default) at fixed positions of the
// concatenated arrays, whatever the tables, and lists per slice the
// (table, begin, end) runs it covers; a slice whose tables' LDS images
// would not fit is split at a table.  The grid's workgroups take the slices
// round-robin (workgroup b: launch positions b, b + grid, ...; the host
// orders the positions so that runs of 8 consecutive slices share an XCD),
// so the workgroups in flight stream neighbouring slices and every slice is
// streamed in full iterations: a slice boundary, not a table boundary, ends
// an iteration.  The forward's grid is persistent (a few workgroups per CU);
// the backward's has about one workgroup per slice.  Per slice a workgroup
// copies its tables' images (one
// contiguous span of the batch's image arena) into LDS, passes a barrier and
// streams the slice as one range; each wave looks up the run of its
// 64 vectors (scalar: the slice's runs are in order) and, where the vectors
// cross a table boundary, evaluates each point with its own table.
//
// Fused backward: the same, in slices of four iterations, with one FP64
// dL/dv region per table of the slice in LDS after the images.  After the
// slice the workgroup stores every region, rounded to FP32, as that run's
// partial sums in a buffer of the batch; k_batch_dv_reduce then adds each
// table's partial sums in slice order, in FP64, so dL/dv does not depend on
// the order in which the workgroups ran.
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

// The first W * blockDim.x words of the next unit's images, loaded into
// registers when the current unit starts, so that their latency passes
// while the current unit streams; put_words writes them (and stages any
// further words) once every wave is done with the current unit.
template <int W>
struct ImagePrefetch {
  v4f w[W];
};

template <int W>
__device__ __forceinline__ void prefetch_words(const float4* __restrict__ src4, int n, ImagePrefetch<W>& p) {
  const v4f* __restrict__ src = reinterpret_cast<const v4f*>(src4);
  const int tid = threadIdx.x, bs = blockDim.x;
#pragma unroll
  for (int j = 0; j < W; ++j) p.w[j] = src[min(j * bs + tid, n - 1)];
}

template <int W>
__device__ __forceinline__ void put_words(const ImagePrefetch<W>& p, const float4* __restrict__ src4, int n,
                                          float4* dst4) {
  v4f* dst = reinterpret_cast<v4f*>(dst4);
  const int tid = threadIdx.x, bs = blockDim.x;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const int k = j * bs + tid;
    if (k < n) dst[k] = p.w[j];
  }
  if (n > W * bs) stage_words(src4 + W * bs, n - W * bs, dst4 + W * bs);
}

// A workgroup barrier that orders LDS accesses only: the streaming stores a
// wave still has in flight are not waited for (__syncthreads would).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Run q of a slice: its points and its table, whose image is in LDS.  q is
// uniform, so the descriptor comes through the scalar cache.
struct RunView {
  EvalTable t;
  Smem s;
  int64_t begin, end;
};

template <bool DV = false>
__device__ __forceinline__ RunView run_view(const BatchRun* __restrict__ runs, int q, float4* lds) {
  const BatchRun r = runs[q];
  RunView v;
  v.t = run_table(r);
  v.s = carve(lds + r.img_lds, r.N, r.K, false);
  if (DV) {
    v.s.dv = reinterpret_cast<double*>(lds + r.dv_lds);
    v.s.dvc = dv_copies(r.N);
  }
  v.begin = r.begin;
  v.end = r.end;
  return v;
}

template <int MAXC>
__device__ __forceinline__ v4f eval4(const v4f& xv, const RunView& v) {
  v4f yv;
  yv.x = eval_point<MAXC>(xv.x, v.t, v.s);
  yv.y = eval_point<MAXC>(xv.y, v.t, v.s);
  yv.z = eval_point<MAXC>(xv.z, v.t, v.s);
  yv.w = eval_point<MAXC>(xv.w, v.t, v.s);
  return yv;
}

// Points [lo, hi) of runs [r0, r1) one by one (the unaligned ends of a
// slice, or every point when the arrays cannot be read as vectors).
template <int MAXC>
__device__ __forceinline__ void slice_scalar(const BatchRun* __restrict__ runs, int r0, int r1, float4* lds,
                                             const float* __restrict__ x, float* __restrict__ y, int64_t lo,
                                             int64_t hi) {
  if (lo >= hi) return;
  for (int q = r0; q < r1; ++q) {
    const RunView v = run_view(runs, q, lds);
    const int64_t a = v.begin > lo ? v.begin : lo, b = v.end < hi ? v.end : hi;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) y[i] = eval_point<MAXC>(x[i], v.t, v.s);
  }
}

// One iteration of a slice: U vectors per thread, vectors ib + tid + u bs.
// Loads, then lookups, then stores, as in the single-table body.  The 64
// vectors of a wave (points pf .. pf + 255) take the run `cur`, advanced to
// the one holding pf; a wave whose points reach past it evaluates each
// point under the run it falls in, for the runs up to the wave's last point.
template <int U, int MAXC, bool GUARD>
__device__ __forceinline__ void slice_iter(const BatchRun* __restrict__ runs, int r1, float4* lds, RunView& cur,
                                           int& q, const v4f* __restrict__ x4, v4f* __restrict__ y4,
                                           int64_t ib, int64_t vend, int64_t phase, int64_t e, int tid,
                                           int wave0) {
  const int64_t bs = blockDim.x;
  v4f xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = ib + tid + u * bs;
    if (!GUARD || i < vend) xv[u] = __builtin_nontemporal_load(x4 + i);
  }
  v4f yv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t w = ib + wave0 + u * bs;   // the wave's first vector
    if (GUARD && w >= vend) continue;       // no lane of the wave has a vector here
    const int64_t pf = 4 * w - phase;
    const int64_t pl = (pf + 255 < e - 1) ? pf + 255 : e - 1;
    while (cur.end <= pf && q + 1 < r1) cur = run_view(runs, ++q, lds);
    if (pl < cur.end) {
      yv[u] = eval4<MAXC>(xv[u], cur);
    } else {
      const int64_t p0 = 4 * (ib + tid + u * bs) - phase;   // this lane's first point
      v4f out = xv[u];
      RunView v = cur;
      for (int qq = q;;) {
        if (p0 >= v.begin && p0 < v.end) out.x = eval_point<MAXC>(xv[u].x, v.t, v.s);
        if (p0 + 1 >= v.begin && p0 + 1 < v.end) out.y = eval_point<MAXC>(xv[u].y, v.t, v.s);
        if (p0 + 2 >= v.begin && p0 + 2 < v.end) out.z = eval_point<MAXC>(xv[u].z, v.t, v.s);
        if (p0 + 3 >= v.begin && p0 + 3 < v.end) out.w = eval_point<MAXC>(xv[u].w, v.t, v.s);
        if (v.end > pl || qq + 1 >= r1) break;
        v = run_view(runs, ++qq, lds);
      }
      yv[u] = out;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = ib + tid + u * bs;
    if (!GUARD || i < vend) __builtin_nontemporal_store(yv[u], y4 + i);
  }
}

// A slice: runs [r0, r1), points [runs[r0].begin, runs[r1-1].end), their
// images staged at the runs' img_lds.
template <int U, int MAXC>
__device__ __forceinline__ void slice_fwd(const BatchRun* __restrict__ runs, int r0, int r1, float4* lds,
                                          const float* __restrict__ x, float* __restrict__ y, bool vec,
                                          int wave0) {
  const int64_t b = runs[r0].begin, e = runs[r1 - 1].end;
  const Split sp = split_range(x, b, e, vec);
  if (sp.vend <= sp.vbeg) {
    slice_scalar<MAXC>(runs, r0, r1, lds, x, y, b, e);
    return;
  }
  const int64_t phase = (int64_t)((reinterpret_cast<uintptr_t>(x) >> 2) & 3);
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x - phase);
  v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y - phase);
  const int tid = threadIdx.x;
  const int64_t chunk = (int64_t)blockDim.x * U;
  int q = r0;
  RunView cur = run_view(runs, q, lds);
  int64_t ib = sp.vbeg;
  for (; ib + chunk <= sp.vend; ib += chunk)
    slice_iter<U, MAXC, false>(runs, r1, lds, cur, q, x4, y4, ib, sp.vend, phase, e, tid, wave0);
  if (ib < sp.vend) slice_iter<U, MAXC, true>(runs, r1, lds, cur, q, x4, y4, ib, sp.vend, phase, e, tid, wave0);
  slice_scalar<MAXC>(runs, r0, r1, lds, x, y, b, sp.head);
  const int64_t tail = 4 * sp.vend - phase;
  slice_scalar<MAXC>(runs, r0, r1, lds, x, y, tail > sp.head ? tail : sp.head, e);
}

// Units blockIdx.x, blockIdx.x + gridDim.x, ...: the first unit's images
// are staged, then per unit: load the next unit's first image words (four
// per thread) into registers, stream this unit, one barrier, write the next
// images to LDS, one barrier.
template <int U>
__global__ __launch_bounds__(1024) void k_batch_fwd(const BatchRun* __restrict__ runs,
                                                    const BatchGroup* __restrict__ groups, int ngroups,
                                                    const float4* __restrict__ arena,
                                                    const float* __restrict__ x, float* __restrict__ y,
                                                    int vec) {
  extern __shared__ float4 lds_f4[];
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;
  int gi = blockIdx.x;
  if (gi >= ngroups) return;
  BatchGroup gp = groups[gi];
  stage_words(arena + gp.img, gp.nwords, lds_f4);
  lds_barrier();
  for (;;) {
    const int gn = gi + (int)gridDim.x;
    const bool more = gn < ngroups;
    BatchGroup gq{};
    ImagePrefetch<4> pf;
    if (more) {
      gq = groups[gn];
      prefetch_words(arena + gq.img, gq.nwords, pf);
    }
    switch (gp.maxc) {
      case 0:
      case 1: slice_fwd<U, 1>(runs, gp.r0, gp.r1, lds_f4, x, y, vec != 0, wave0); break;
      case 2: slice_fwd<U, 2>(runs, gp.r0, gp.r1, lds_f4, x, y, vec != 0, wave0); break;
      case 3: slice_fwd<U, 3>(runs, gp.r0, gp.r1, lds_f4, x, y, vec != 0, wave0); break;
      case 4: slice_fwd<U, 4>(runs, gp.r0, gp.r1, lds_f4, x, y, vec != 0, wave0); break;
      default: slice_fwd<U, 0>(runs, gp.r0, gp.r1, lds_f4, x, y, vec != 0, wave0); break;
    }
    if (!more) break;
    lds_barrier();
    put_words(pf, arena + gq.img, gq.nwords, lds_f4);
    lds_barrier();
    gi = gn;
    gp = gq;
  }
}

// The fused backward of a slice, as slice_fwd: x and g in, y and dx out
// (each optional), every point's two hat weights into its run's FP64 dL/dv
// region in LDS.  Lanes past the slice's vectors take no point (their
// weights would be added).
template <int MAXC, bool WY, bool WDX>
__device__ __forceinline__ void bwd_point(float xv, float gv, const RunView& v, float& yv, float& dxv) {
  backward_point<MAXC, WY, WDX, true>(xv, gv, v.t, v.s, yv, dxv);
}

template <int MAXC, bool WY, bool WDX>
__device__ __forceinline__ void slice_bwd_scalar(const BatchRun* __restrict__ runs, int r0, int r1, float4* lds,
                                                 const float* __restrict__ x, const float* __restrict__ g,
                                                 float* __restrict__ y, float* __restrict__ dx, int64_t lo,
                                                 int64_t hi) {
  if (lo >= hi) return;
  for (int q = r0; q < r1; ++q) {
    const RunView v = run_view<true>(runs, q, lds);
    const int64_t a = v.begin > lo ? v.begin : lo, b = v.end < hi ? v.end : hi;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
      float yy = 0.0f, dd = 0.0f;
      bwd_point<MAXC, WY, WDX>(x[i], g[i], v, yy, dd);
      if (WY) y[i] = yy;
      if (WDX) dx[i] = dd;
    }
  }
}

template <int U, int MAXC, bool GUARD, bool WY, bool WDX>
__device__ __forceinline__ void slice_bwd_iter(const BatchRun* __restrict__ runs, int r1, float4* lds,
                                               RunView& cur, int& q, const v4f* __restrict__ x4,
                                               const v4f* __restrict__ g4, v4f* __restrict__ y4,
                                               v4f* __restrict__ dx4, int64_t ib, int64_t vend, int64_t phase,
                                               int64_t e, int tid, int wave0) {
  const int64_t bs = blockDim.x;
  v4f xv[U], gv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = ib + tid + u * bs;
    if (!GUARD || i < vend) {
      xv[u] = __builtin_nontemporal_load(x4 + i);
      gv[u] = __builtin_nontemporal_load(g4 + i);
    }
  }
  v4f yv[U], dxv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t w = ib + wave0 + u * bs;
    if (GUARD && w >= vend) continue;
    const int64_t pf = 4 * w - phase;
    const int64_t pl = (pf + 255 < e - 1) ? pf + 255 : e - 1;
    while (cur.end <= pf && q + 1 < r1) cur = run_view<true>(runs, ++q, lds);
    if (GUARD && ib + tid + u * bs >= vend) continue;   // this lane has no vector here
    float yy = 0.0f, dd = 0.0f;
    if (pl < cur.end) {
      bwd_point<MAXC, WY, WDX>(xv[u].x, gv[u].x, cur, yy, dd); yv[u].x = yy; dxv[u].x = dd;
      bwd_point<MAXC, WY, WDX>(xv[u].y, gv[u].y, cur, yy, dd); yv[u].y = yy; dxv[u].y = dd;
      bwd_point<MAXC, WY, WDX>(xv[u].z, gv[u].z, cur, yy, dd); yv[u].z = yy; dxv[u].z = dd;
      bwd_point<MAXC, WY, WDX>(xv[u].w, gv[u].w, cur, yy, dd); yv[u].w = yy; dxv[u].w = dd;
    } else {
      const int64_t p0 = 4 * (ib + tid + u * bs) - phase;
      RunView v = cur;
      for (int qq = q;;) {
        if (p0 >= v.begin && p0 < v.end) { bwd_point<MAXC, WY, WDX>(xv[u].x, gv[u].x, v, yy, dd); yv[u].x = yy; dxv[u].x = dd; }
        if (p0 + 1 >= v.begin && p0 + 1 < v.end) { bwd_point<MAXC, WY, WDX>(xv[u].y, gv[u].y, v, yy, dd); yv[u].y = yy; dxv[u].y = dd; }
        if (p0 + 2 >= v.begin && p0 + 2 < v.end) { bwd_point<MAXC, WY, WDX>(xv[u].z, gv[u].z, v, yy, dd); yv[u].z = yy; dxv[u].z = dd; }
        if (p0 + 3 >= v.begin && p0 + 3 < v.end) { bwd_point<MAXC, WY, WDX>(xv[u].w, gv[u].w, v, yy, dd); yv[u].w = yy; dxv[u].w = dd; }
        if (v.end > pl || qq + 1 >= r1) break;
        v = run_view<true>(runs, ++qq, lds);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = ib + tid + u * bs;
    if (!GUARD || i < vend) {
      if (WY) __builtin_nontemporal_store(yv[u], y4 + i);
      if (WDX) __builtin_nontemporal_store(dxv[u], dx4 + i);
    }
  }
}

template <int U, int MAXC, bool WY, bool WDX>
__device__ __forceinline__ void slice_bwd(const BatchRun* __restrict__ runs, int r0, int r1, float4* lds,
                                          const float* __restrict__ x, const float* __restrict__ g,
                                          float* __restrict__ y, float* __restrict__ dx, bool vec, int wave0) {
  const int64_t b = runs[r0].begin, e = runs[r1 - 1].end;
  const Split sp = split_range(x, b, e, vec);
  if (sp.vend <= sp.vbeg) {
    slice_bwd_scalar<MAXC, WY, WDX>(runs, r0, r1, lds, x, g, y, dx, b, e);
    return;
  }
  const int64_t phase = (int64_t)((reinterpret_cast<uintptr_t>(x) >> 2) & 3);
  const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x - phase);
  const v4f* __restrict__ g4 = reinterpret_cast<const v4f*>(g - phase);
  v4f* __restrict__ y4 = WY ? reinterpret_cast<v4f*>(y - phase) : nullptr;
  v4f* __restrict__ dx4 = WDX ? reinterpret_cast<v4f*>(dx - phase) : nullptr;
  const int tid = threadIdx.x;
  const int64_t chunk = (int64_t)blockDim.x * U;
  int q = r0;
  RunView cur = run_view<true>(runs, q, lds);
  int64_t ib = sp.vbeg;
  for (; ib + chunk <= sp.vend; ib += chunk)
    slice_bwd_iter<U, MAXC, false, WY, WDX>(runs, r1, lds, cur, q, x4, g4, y4, dx4, ib, sp.vend, phase, e, tid,
                                            wave0);
  if (ib < sp.vend)
    slice_bwd_iter<U, MAXC, true, WY, WDX>(runs, r1, lds, cur, q, x4, g4, y4, dx4, ib, sp.vend, phase, e, tid,
                                           wave0);
  slice_bwd_scalar<MAXC, WY, WDX>(runs, r0, r1, lds, x, g, y, dx, b, sp.head);
  const int64_t tail = 4 * sp.vend - phase;
  slice_bwd_scalar<MAXC, WY, WDX>(runs, r0, r1, lds, x, g, y, dx, tail > sp.head ? tail : sp.head, e);
}

// As k_batch_fwd, with the unit's FP64 dL/dv regions (one per table, after
// the images) zeroed before the barrier that starts it; after the unit, one
// more barrier and every region is stored, rounded to FP32, as its run's
// partial sums (k_batch_dv_reduce adds them up), then one more barrier
// before the next unit's images overwrite LDS.  Two image words per thread
// are prefetched (four would spill: the backward holds twice the data).
template <int U, bool WY, bool WDX>
__global__ __launch_bounds__(1024) void k_batch_bwd(const BatchRun* __restrict__ runs,
                                                    const BatchGroup* __restrict__ groups, int ngroups,
                                                    const float4* __restrict__ arena,
                                                    const float* __restrict__ x, const float* __restrict__ g,
                                                    float* __restrict__ y, float* __restrict__ dx,
                                                    float* __restrict__ part, int vec) {
  extern __shared__ float4 lds_f4[];
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;
  int gi = blockIdx.x;
  if (gi >= ngroups) return;
  BatchGroup gp = groups[gi];
  stage_words(arena + gp.img, gp.nwords, lds_f4);
  for (;;) {
    double* dvz = reinterpret_cast<double*>(lds_f4 + gp.dv_lds);
    for (int k = threadIdx.x; k < 2 * gp.dv_words; k += blockDim.x) dvz[k] = 0.0;
    lds_barrier();
    const int gn = gi + (int)gridDim.x;
    const bool more = gn < ngroups;
    BatchGroup gq{};
    ImagePrefetch<2> pf;
    if (more) {
      gq = groups[gn];
      prefetch_words(arena + gq.img, gq.nwords, pf);
    }
    switch (gp.maxc) {
      case 0:
      case 1: slice_bwd<U, 1, WY, WDX>(runs, gp.r0, gp.r1, lds_f4, x, g, y, dx, vec != 0, wave0); break;
      case 2: slice_bwd<U, 2, WY, WDX>(runs, gp.r0, gp.r1, lds_f4, x, g, y, dx, vec != 0, wave0); break;
      case 3: slice_bwd<U, 3, WY, WDX>(runs, gp.r0, gp.r1, lds_f4, x, g, y, dx, vec != 0, wave0); break;
      case 4: slice_bwd<U, 4, WY, WDX>(runs, gp.r0, gp.r1, lds_f4, x, g, y, dx, vec != 0, wave0); break;
      default: slice_bwd<U, 0, WY, WDX>(runs, gp.r0, gp.r1, lds_f4, x, g, y, dx, vec != 0, wave0); break;
    }
    lds_barrier();
    for (int q = gp.r0; q < gp.r1; ++q) {
      const BatchRun r = runs[q];
      const double* d = reinterpret_cast<const double*>(lds_f4 + r.dv_lds);
      const int c = dv_copies(r.N);
      float* out = part + r.part;
      for (int k = threadIdx.x; k <= r.N; k += blockDim.x) {
        double acc = d[k * c];
        for (int j = 1; j < c; ++j) acc += d[k * c + j];   // copies in a fixed order
        out[k] = (float)acc;
      }
    }
    if (!more) break;
    lds_barrier();
    put_words(pf, arena + gq.img, gq.nwords, lds_f4);
    gi = gn;
    gp = gq;
  }
}

// dL/dv of table blockIdx.x, entries 256 blockIdx.y + threadIdx.x: each the
// sum, in FP64 and in slice order (a fixed order: the result does not depend
// on how the workgroups ran), of its runs' partial sums; zero for a table
// without points.  Writes every entry of dv.
__global__ __launch_bounds__(256) void k_batch_dv_reduce(const float* __restrict__ part,
                                                         const int64_t* __restrict__ tab_part,
                                                         const int32_t* __restrict__ tab_first,
                                                         const int64_t* __restrict__ tab_dv,
                                                         float* __restrict__ dv) {
  const int t = blockIdx.x;
  const int64_t d0 = tab_dv[t], n1 = tab_dv[t + 1] - d0;
  const int j0 = tab_first[t], j1 = tab_first[t + 1];
  const int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (k < n1) {
    double acc = 0.0;
    int j = j0;
    for (; j + 8 <= j1; j += 8) {   // eight loads in flight, added in order
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[tab_part[j + q] + k];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += (double)v[q];
    }
    for (; j < j1; ++j) acc += (double)part[tab_part[j] + k];
    dv[d0 + k] = (float)acc;
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

inline bool same_phase(const void* a, const void* b) {
  return b == nullptr || ((reinterpret_cast<uintptr_t>(a) ^ reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
}

hipError_t launch_plan(const BatchLaunch& bl, const BatchPlan& p, const LaunchConfig& c, const float* x,
                       const float* g, float* y, float* dx, int v, hipStream_t s) {
  const dim3 grid(p.grid), block(c.block);
  if (g == nullptr) {
    switch (c.unroll) {
      case 1: hipLaunchKernelGGL(k_batch_fwd<1>, grid, block, p.lds, s, p.runs, p.groups, p.ngroups, p.arena, x, y, v); break;
      case 2: hipLaunchKernelGGL(k_batch_fwd<2>, grid, block, p.lds, s, p.runs, p.groups, p.ngroups, p.arena, x, y, v); break;
      default: hipLaunchKernelGGL(k_batch_fwd<4>, grid, block, p.lds, s, p.runs, p.groups, p.ngroups, p.arena, x, y, v); break;
    }
    return hipGetLastError();
  }
  const int key = (y != nullptr ? 2 : 0) | (dx != nullptr ? 1 : 0);
#define PWL_BB(UU, A, B)                                                                              \
  hipLaunchKernelGGL((k_batch_bwd<UU, A, B>), grid, block, p.lds, s, p.runs, p.groups, p.ngroups, p.arena, x, g, \
                     y, dx, bl.part, v)
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
  const hipError_t e = launch_plan(bl, backward ? bl.bwd : bl.fwd, c, x, g, y, dx, v, s);
  if (e != hipSuccess || !backward) return e;
  hipLaunchKernelGGL(k_batch_dv_reduce, dim3((unsigned)bl.T, (unsigned)((bl.max_n + 256) / 256)), dim3(256), 0, s,
                     bl.part, bl.tab_part, bl.tab_first, bl.tab_dv, dv);
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
