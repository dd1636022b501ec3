// Device building blocks of the streaming evaluators (single-table and
// batched): the LDS image of a table, the segment locate, one point of
// Algorithm 1 and of its derivative, and one grid-stride iteration over U
// float4 vectors per thread.
#pragma once

#include <hip/hip_runtime.h>

#include "pwl_internal.h"
#include "pwl_locate.h"

namespace pwl {
namespace stream {

typedef float v4f __attribute__((ext_vector_type(4)));

// Packed records: one 16-byte word per segment (a segment's lookup is one
// LDS read of 12 or 16 bytes).
struct Smem {
  float4* rec;      // [N]           {x_k, v_k, slope_k, x_{k+1}}
  float* knot;      // [N + pad]     knot[k] = x_k for 1 <= k <= N-1, NaN elsewhere
  uint16_t* lo;     // [K + 1]       lo[u] = #{interior knots in cells < u}; lo[K] = N - 1
  double* dv;       // [(N + 1) dvc] backward only: this workgroup's dL/dv, entry k of copy c at k dvc + c
  int dvc;          //               copies of dL/dv (a power of two; lane l adds into copy l mod dvc)
  __device__ __forceinline__ float4 record(int k) const { return rec[k]; }
  __device__ __forceinline__ void put_record(int k, float4 r) const { rec[k] = r; }
};

// Structure-of-arrays records: the four fields of the records in four
// arrays of N floats (a lookup reads each field it uses separately; the
// forward's three reads are 4 bytes each).  Forward evaluation only.
struct SmemSoA {
  float* rx;        // [N] x_k
  float* rv;        // [N] v_k
  float* rs;        // [N] slope_k
  float* rw;        // [N] x_{k+1}
  float* knot;
  uint16_t* lo;
  __device__ __forceinline__ float4 record(int k) const { return make_float4(rx[k], rv[k], rs[k], rw[k]); }
  __device__ __forceinline__ void put_record(int k, float4 r) const {
    rx[k] = r.x;
    rv[k] = r.y;
    rs[k] = r.z;
    rw[k] = r.w;
  }
};

// Value/slope pairs: one 8-byte pair {v_k, slope_k} per segment, with x_k
// read from the knot array, whose entry 0 holds a (no compare reads entry 0,
// so it can): a point reads its map cell, the knots of its cell with the one
// before them (the segment's own knot among them; adjacent, so one paired
// read for a cell of one knot) and one pair.  Forward evaluation only.
struct SmemPairs {
  float2* vs;       // [N]        {v_k, slope_k}
  float* knot;      // [N + pad]  knot[0] = a, knot[k] = x_k for 1 <= k <= N-1, NaN from N on
  uint16_t* lo;
};

// Sections of a table image (see image_words).  Every pointer is an offset
// from `base` itself: a pointer rebuilt from an integer would lose its
// address space, and LDS accesses (the dL/dv atomics above all) would go
// through the flat path.
__device__ __forceinline__ Smem carve(void* base, int N, int K, bool backward) {
  Smem s;
  s.rec = reinterpret_cast<float4*>(base);
  s.knot = reinterpret_cast<float*>(s.rec + N);
  s.lo = reinterpret_cast<uint16_t*>(reinterpret_cast<float4*>(s.knot) + image_knot_words(N));
  s.dv = backward ? reinterpret_cast<double*>(reinterpret_cast<float4*>(s.lo) + image_map_words(K)) : nullptr;
  s.dvc = backward ? dv_copies(N) : 1;
  return s;
}

// The structure-of-arrays image: four record arrays of image_soa_field_words
// words each, then the knots and the map as in carve.
__device__ __forceinline__ SmemSoA carve_soa(void* base, int N, int K) {
  SmemSoA s;
  const int fw = image_soa_field_words(N);
  float4* b4 = reinterpret_cast<float4*>(base);
  s.rx = reinterpret_cast<float*>(b4);
  s.rv = reinterpret_cast<float*>(b4 + fw);
  s.rs = reinterpret_cast<float*>(b4 + 2 * fw);
  s.rw = reinterpret_cast<float*>(b4 + 3 * fw);
  s.knot = reinterpret_cast<float*>(b4 + 4 * fw);
  s.lo = reinterpret_cast<uint16_t*>(reinterpret_cast<float4*>(s.knot) + image_knot_words(N));
  (void)K;
  return s;
}

// The pairs image: the pairs (two per 16-byte word), then the knots and the
// map as in carve.
__device__ __forceinline__ SmemPairs carve_pairs(void* base, int N, int K) {
  SmemPairs s;
  float4* b4 = reinterpret_cast<float4*>(base);
  s.vs = reinterpret_cast<float2*>(b4);
  s.knot = reinterpret_cast<float*>(b4 + image_pair_words(N));
  s.lo = reinterpret_cast<uint16_t*>(reinterpret_cast<float4*>(s.knot) + image_knot_words(N));
  (void)K;
  return s;
}

// The words of the table's image (see image_words; the table's arrays are
// 256-byte aligned).  A record, with v_override its value and slope
// re-derived as (v_{k+1} - v_k) / (x_{k+1} - x_k) in FP32:
__device__ __forceinline__ float4 record_word(const EvalTable& t, const float* __restrict__ vo, int w) {
  float4 r = t.rec[w];
  if (vo != nullptr) {
    const float v0 = vo[w], v1 = vo[w + 1];
    r.y = v0;
    r.z = (v1 - v0) / (r.w - r.x);
  }
  return r;
}

// knots 4w .. 4w+3, NaN outside the interior knots 1..N-1 (so that every
// compare against a sentinel is false, even for x = +inf):
__device__ __forceinline__ float4 knot_word(const EvalTable& t, int w) {
  const int k0 = 4 * w;
  if (k0 >= 1 && k0 + 3 <= t.N - 1) return *reinterpret_cast<const float4*>(t.knots + k0);
  float e[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = k0 + i;
    e[i] = (k >= 1 && k <= t.N - 1) ? t.knots[k] : __builtin_nanf("");
  }
  return make_float4(e[0], e[1], e[2], e[3]);
}

// The same with entry 0 = a (the pairs image):
__device__ __forceinline__ float4 knot_word_a(const EvalTable& t, int w) {
  float4 k = knot_word(t, w);
  if (w == 0) k.x = t.a32;
  return k;
}

// map entries 8w .. 8w+7, 0 past lo[K]:
__device__ __forceinline__ float4 map_word(const EvalTable& t, int w) {
  const int u0 = 8 * w;
  if (u0 + 7 <= t.K) return *reinterpret_cast<const float4*>(t.lo + u0);
  uint32_t p[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int u = u0 + 2 * i;
    const uint32_t lo = (u <= t.K) ? t.lo[u] : 0u, hi = (u + 1 <= t.K) ? t.lo[u + 1] : 0u;
    p[i] = lo | (hi << 16);
  }
  return make_float4(__uint_as_float(p[0]), __uint_as_float(p[1]), __uint_as_float(p[2]), __uint_as_float(p[3]));
}

// Copy the table's image to `s` (LDS, or a batch's image in global memory).
// When every section fits in one word per thread (N no larger than the
// workgroup), each thread loads its words before it writes any, so the copy
// waits on one round of loads instead of one per section; the straight-line
// form keeps the kernels' register use where the streaming loop needs it.
template <class S>
__device__ __forceinline__ void stage_table(const EvalTable& t, const float* __restrict__ vo, const S& s) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nkw = image_knot_words(t.N), nmw = image_map_words(t.K);
  float4* knot4 = reinterpret_cast<float4*>(s.knot);
  float4* map4 = reinterpret_cast<float4*>(s.lo);
  if (t.N <= nt && nkw <= nt && nmw <= nt) {
    const bool hr = tid < t.N, hk = tid < nkw, hm = tid < nmw;
    float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f), k = r, m = r;
    if (hr) r = record_word(t, vo, tid);
    if (hk) k = knot_word(t, tid);
    if (hm) m = map_word(t, tid);
    if (hr) s.put_record(tid, r);
    if (hk) knot4[tid] = k;
    if (hm) map4[tid] = m;
    return;
  }
  for (int w = tid; w < t.N; w += nt) s.put_record(w, record_word(t, vo, w));
  for (int w = tid; w < nkw; w += nt) knot4[w] = knot_word(t, w);
  for (int w = tid; w < nmw; w += nt) map4[w] = map_word(t, w);
}

// The pairs image: word w holds the pairs of segments 2w and 2w + 1 (zero
// past N - 1); sections as in stage_table, each in one round of loads when
// it fits in one word per thread.
__device__ __forceinline__ float4 pair_word(const EvalTable& t, const float* __restrict__ vo, int w) {
  const float4 r0 = record_word(t, vo, 2 * w);
  float4 r1 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (2 * w + 1 < t.N) r1 = record_word(t, vo, 2 * w + 1);
  return make_float4(r0.y, r0.z, r1.y, r1.z);
}

__device__ __forceinline__ void stage_table_pairs(const EvalTable& t, const float* __restrict__ vo,
                                                  const SmemPairs& s) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int npw = image_pair_words(t.N), nkw = image_knot_words(t.N), nmw = image_map_words(t.K);
  float4* pair4 = reinterpret_cast<float4*>(s.vs);
  float4* knot4 = reinterpret_cast<float4*>(s.knot);
  float4* map4 = reinterpret_cast<float4*>(s.lo);
  if (npw <= nt && nkw <= nt && nmw <= nt) {
    const bool hp = tid < npw, hk = tid < nkw, hm = tid < nmw;
    float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f), k = p, m = p;
    if (hp) p = pair_word(t, vo, tid);
    if (hk) k = knot_word_a(t, tid);
    if (hm) m = map_word(t, tid);
    if (hp) pair4[tid] = p;
    if (hk) knot4[tid] = k;
    if (hm) map4[tid] = m;
    return;
  }
  for (int w = tid; w < npw; w += nt) pair4[w] = pair_word(t, vo, w);
  for (int w = tid; w < nkw; w += nt) knot4[w] = knot_word_a(t, w);
  for (int w = tid; w < nmw; w += nt) map4[w] = map_word(t, w);
}

__device__ __forceinline__ float clamp_nan(float x, float a, float b) {
  return (x < a) ? a : ((x > b) ? b : x);   // NaN passes through
}

// Segment of x when no map cell holds more than MAXC knots: compare x with
// the MAXC knots that follow lo[cell(x)].  Knots beyond the cell's own are
// greater than x (they lie in later cells) and the sentinels are NaN, so the
// extra compares are false; the count of true compares is exact.
template <int MAXC, class S>
__device__ __forceinline__ int locate_fixed(float x, const EvalTable& t, const S& s) {
  const int u = map_cell(x, t.a32, t.scale32, t.K);
  const int lo = s.lo[u];
  int seg = lo;
#pragma unroll
  for (int j = 1; j <= MAXC; ++j) seg += (x >= s.knot[lo + j]) ? 1 : 0;
  return seg;
}

// Any number of knots per cell: the count is lo[u+1] - lo[u].
template <class S>
__device__ __forceinline__ int locate_any(float x, const EvalTable& t, const S& s) {
  const int u = map_cell(x, t.a32, t.scale32, t.K);
  const int lo = s.lo[u];
  const int cnt = (int)s.lo[u + 1] - lo;
  int seg = lo;
  for (int j = 1; j <= cnt; ++j) seg += (x >= s.knot[lo + j]) ? 1 : 0;
  return seg;
}

// The paper's GPU locate (Sec. IV-V): a branch-free binary search over the
// knots, here the interior knots in LDS.  It counts the interior knots <= x
// (so x_i <= x < x_{i+1}; NaN x compares false and gives 0), halving a
// power-of-two step from the largest one below N.
template <class S>
__device__ __forceinline__ int locate_search(float x, const EvalTable& t, const S& s) {
  int lo = 0;
  for (int half = (t.N > 1) ? (1 << (31 - __builtin_clz(t.N - 1))) : 0; half >= 1; half >>= 1) {
    const int k = lo + half;
    lo = (k < t.N && s.knot[k] <= x) ? k : lo;
  }
  return lo;
}

// MAXC > 0: map + MAXC unrolled compares; 0: map + counted compares;
// -1: binary search without the map.
template <int MAXC, class S>
__device__ __forceinline__ int locate(float x, const EvalTable& t, const S& s) {
  if (MAXC > 0) return locate_fixed<MAXC>(x, t, s);
  if (MAXC < 0) return locate_search(x, t, s);
  return locate_any(x, t, s);
}

template <int MAXC, class S>
__device__ __forceinline__ float eval_point(float x, const EvalTable& t, const S& s) {
  const int seg = locate<MAXC>(x, t, s);
  const float4 r = s.record(seg);
  return fmaf(clamp_nan(x, t.a32, t.b32) - r.x, r.z, r.y);
}

// Algorithm 1 through the pairs image.  With MAXC unrolled compares the
// segment's knot comes out of the compares themselves (the last knot of the
// cell that x reaches, or the knot before the cell), so the knot reads are
// adjacent; otherwise it is read after the locate.  The same operations on
// the same values as eval_point, so the outputs are bit-identical.
template <int MAXC>
__device__ __forceinline__ float eval_point(float x, const EvalTable& t, const SmemPairs& s) {
  int seg;
  float xs;
  if (MAXC > 0) {
    const int u = map_cell(x, t.a32, t.scale32, t.K);
    const int lo = s.lo[u];
    seg = lo;
    xs = s.knot[lo];
#pragma unroll
    for (int j = 1; j <= MAXC; ++j) {
      const float kj = s.knot[lo + j];
      const bool c = x >= kj;
      seg += c ? 1 : 0;
      xs = c ? kj : xs;
    }
  } else {
    seg = locate<MAXC>(x, t, s);
    xs = s.knot[seg];
  }
  const float2 p = s.vs[seg];
  return fmaf(clamp_nan(x, t.a32, t.b32) - xs, p.y, p.x);
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
      // Each hat weight comes from its own knot distance, (x_{k+1} - x)/h and
      // (x - x_k)/h, with x_{k+1} from the record: forming (1 - delta) g as
      // g - delta g would cancel when delta is near 1.
      const float xc = clamp_nan(x, t.a32, t.b32);
      const float rh = __builtin_amdgcn_rcpf(r.w - r.x);   // 1/h, within 1 ulp
      const float w0 = ((r.w - xc) * rh) * g;   // (1 - delta) g
      const float w1 = (d * rh) * g;            // delta g
      const int at = seg * s.dvc + ((int)__lane_id() & (s.dvc - 1));
      __hip_atomic_fetch_add(s.dv + at, (double)w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(s.dv + at + s.dvc, (double)w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// One iteration over U float4 vectors per thread: all loads, then all table
// lookups, then all stores.  Full iterations run unguarded so the compiler
// can count outstanding memory operations exactly (a guarded load makes
// every later wait a wait for all stores); the last, partial iteration of a
// thread is guarded.
template <int U, int MAXC, bool GUARD, class S>
__device__ __forceinline__ void fwd_iter(const EvalTable& t, const S& s, const v4f* __restrict__ x4,
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

// Which points of [begin, end) go through 16-byte vectors: the arrays share
// their alignment phase (vec), so [head, 4 vend) is vectorised and the
// points before `head` and from max(head, 4 vend) on are scalar.
struct Split {
  int64_t head, vbeg, vend;
};

__device__ __forceinline__ Split split_range(const float* p, int64_t begin, int64_t end, bool vec) {
  Split r;
  if (!vec) {
    r.head = end;
    r.vbeg = r.vend = 0;
    return r;
  }
  // element index whose address is 16-byte aligned, at or after begin
  const int64_t phase = (int64_t)((reinterpret_cast<uintptr_t>(p) >> 2) & 3);
  int64_t h = begin + ((4 - ((phase + begin) & 3)) & 3);
  if (h > end) h = end;
  r.head = h;
  r.vbeg = (phase + h) >> 2;               // in units of the aligned float4 array
  r.vend = (phase + end) >> 2;
  if (r.vend < r.vbeg) r.vend = r.vbeg;
  return r;
}

// Forward over points [begin, end) by `nblk` cooperating workgroups (this one
// is number `blk`): workgroup blk streams vectors blk*bs*U + u*bs + tid of
// each stride of nblk*bs*U vectors.
template <int U, int MAXC, class S>
__device__ __forceinline__ void fwd_range(const EvalTable& t, const S& s, const float* __restrict__ x,
                                          float* __restrict__ y, int64_t begin, int64_t end, bool vec,
                                          int64_t blk, int64_t nblk) {
  const Split sp = split_range(x, begin, end, vec);
  const int64_t bs = blockDim.x, tid = threadIdx.x;
  const int64_t gtid = blk * bs + tid, gthreads = nblk * bs;
  for (int64_t i = begin + gtid; i < sp.head; i += gthreads) y[i] = eval_point<MAXC>(x[i], t, s);
  if (sp.vend > sp.vbeg) {
    const int64_t phase = (int64_t)((reinterpret_cast<uintptr_t>(x) >> 2) & 3);
    const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x - phase);
    v4f* __restrict__ y4 = reinterpret_cast<v4f*>(y - phase);
    const int64_t stride = nblk * bs * U;
    int64_t base = sp.vbeg + blk * bs * U + tid;
    for (; base + (U - 1) * bs < sp.vend; base += stride) fwd_iter<U, MAXC, false>(t, s, x4, y4, base, bs, sp.vend);
    if (base < sp.vend) fwd_iter<U, MAXC, true>(t, s, x4, y4, base, bs, sp.vend);
  }
  const int64_t tail = (sp.vend > sp.vbeg) ? 4 * sp.vend - (int64_t)((reinterpret_cast<uintptr_t>(x) >> 2) & 3)
                                           : sp.head;
  for (int64_t i = (tail > sp.head ? tail : sp.head) + gtid; i < end; i += gthreads)
    y[i] = eval_point<MAXC>(x[i], t, s);
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

  // Fused forward + backward over points [begin, end), cooperating
  // workgroups as in fwd_range.
  template <int MAXC>
  __device__ __forceinline__ static void range(const EvalTable& t, const Smem& s,
                                               const float* __restrict__ x, const float* __restrict__ g,
                                               float* __restrict__ y, float* __restrict__ dx, int64_t begin,
                                               int64_t end, bool vec, int64_t blk, int64_t nblk) {
    const Split sp = split_range(x, begin, end, vec);
    const int64_t bs = blockDim.x, tid = threadIdx.x;
    const int64_t gtid = blk * bs + tid, gthreads = nblk * bs;
    for (int64_t i = begin + gtid; i < sp.head; i += gthreads) scalar<MAXC>(t, s, x, g, y, dx, i);
    const int64_t phase = (int64_t)((reinterpret_cast<uintptr_t>(x) >> 2) & 3);
    if (sp.vend > sp.vbeg) {
      const v4f* __restrict__ x4 = reinterpret_cast<const v4f*>(x - phase);
      const v4f* __restrict__ g4 = reinterpret_cast<const v4f*>(g - phase);
      v4f* __restrict__ y4 = WY ? reinterpret_cast<v4f*>(y - phase) : nullptr;
      v4f* __restrict__ dx4 = WDX ? reinterpret_cast<v4f*>(dx - phase) : nullptr;
      const int64_t stride = nblk * bs * U;
      int64_t base = sp.vbeg + blk * bs * U + tid;
      for (; base + (U - 1) * bs < sp.vend; base += stride)
        iter<MAXC, false>(t, s, x4, g4, y4, dx4, base, bs, sp.vend);
      if (base < sp.vend) iter<MAXC, true>(t, s, x4, g4, y4, dx4, base, bs, sp.vend);
    }
    const int64_t tail = (sp.vend > sp.vbeg) ? 4 * sp.vend - phase : sp.head;
    for (int64_t i = (tail > sp.head ? tail : sp.head) + gtid; i < end; i += gthreads)
      scalar<MAXC>(t, s, x, g, y, dx, i);
  }

  template <int MAXC>
  __device__ __forceinline__ static void scalar(const EvalTable& t, const Smem& s, const float* __restrict__ x,
                                                const float* __restrict__ g, float* __restrict__ y,
                                                float* __restrict__ dx, int64_t i) {
    float yy = 0.0f, dd = 0.0f;
    backward_point<MAXC, WY, WDX, WDV>(x[i], g[i], t, s, yy, dd);
    if (WY) y[i] = yy;
    if (WDX) dx[i] = dd;
  }
};

}  // namespace stream
}  // namespace pwl
