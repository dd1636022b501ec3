// Table construction on the GPU.
//
//   optimal partition (Sec. III-B1):
//     k_density_totals   FP64 |f''|^(2/5) on the fine grid, trapezoid sums per workgroup
//     k_invert_knots     FP64 prefix of those sums, targets i S_M / N, linear inversion
//   every table:
//     k_segments         uniform knots (Sec. IV) if asked; map cell of every knot;
//                        FP32 vertex values f(x_k) (Sec. II-B1) or FP32 Gauss-Legendre
//                        integrals of f against both hats of each segment (Sec. II-B2)
//     k_finalize         one workgroup: the uniform index map, the FP64 solve of
//                        M c = b (parallel cyclic reduction), knot-collapse check and
//                        the packed records {x_k, v_k, slope_k, 1/h_k}
#include <hip/hip_runtime.h>

#include "pwl_func.h"
#include "pwl_internal.h"
#include "pwl_locate.h"

namespace pwl {

namespace {

// Inclusive trapezoid sums of the density over the cells of workgroup `blk`.
// Cell j (1-based) spans [t_{j-1}, t_j], t_j = a + j dt, and adds
// (d_{j-1} + d_j) dt / 2.  Each thread sums its 4 cells sequentially and the
// thread totals are chained sequentially by thread 0, so the sums are
// monotone non-decreasing and the block total equals the last sum bit for
// bit; both kernels below call this same code.  Contraction is off so that
// every operation is one IEEE-rounded FP64 operation.
__device__ double scan_block_cells(const BuildParams& bp, int blk, double* s_d, double* s_tp,
                                   double* s_S) {
#pragma clang fp contract(off)
  constexpr int C = kDensityCellsPerBlock;
  const int tid = threadIdx.x;
  const double dt = (bp.b - bp.a) / (double)bp.M;
  const double hdt = dt / 2.0;
  const int j0 = blk * C;
  for (int s = tid; s <= C; s += kBuildThreads) {
    const int j = j0 + s;
    s_d[s] = (j <= bp.M) ? knot_density(bp.f, bp.a + (double)j * dt) : 0.0;
  }
  __syncthreads();
  double loc[C / kBuildThreads];
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < C / kBuildThreads; ++q) {
    const int c = tid * (C / kBuildThreads) + q;
    const double inc = (j0 + c + 1 <= bp.M) ? (s_d[c] + s_d[c + 1]) * hdt : 0.0;
    acc = acc + inc;
    loc[q] = acc;
  }
  s_tp[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double run = 0.0;
    for (int t = 0; t < kBuildThreads; ++t) {
      const double v = s_tp[t];
      s_tp[t] = run;
      run = run + v;
    }
    s_tp[kBuildThreads] = run;
  }
  __syncthreads();
  if (s_S != nullptr) {
    const double P = s_tp[tid];
#pragma unroll
    for (int q = 0; q < C / kBuildThreads; ++q) s_S[tid * (C / kBuildThreads) + q] = P + loc[q];
  }
  const double total = s_tp[kBuildThreads];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kBuildThreads) void k_density_totals(BuildParams bp, TableDev td) {
  __shared__ double s_d[kDensityCellsPerBlock + 1];
  __shared__ double s_tp[kBuildThreads + 1];
  const double tot = scan_block_cells(bp, blockIdx.x, s_d, s_tp, nullptr);
  if (threadIdx.x == 0) {
    td.totals[blockIdx.x] = tot;
    if (blockIdx.x == 0) *td.status = 0u;
  }
}

__device__ void write_uniform_knots(const BuildParams& bp, const TableDev& td, int k) {
#pragma clang fp contract(off)
  double x = bp.a + ((bp.b - bp.a) * (double)k) / (double)bp.N;
  if (k == 0) x = bp.a;
  if (k == bp.N) x = bp.b;
  td.knots64[k] = x;
  td.knots[k] = (float)x;
}

__global__ __launch_bounds__(kBuildThreads) void k_invert_knots(BuildParams bp, TableDev td) {
#pragma clang fp contract(off)
  constexpr int C = kDensityCellsPerBlock;
  __shared__ double s_d[C + 1];
  __shared__ double s_S[C];
  __shared__ double s_tp[kBuildThreads + 1];
  __shared__ double s_off[3];   // offset of this block, offset of the next, S_M
  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  if (tid == 0) {
    double run = 0.0, off = 0.0, next = 0.0;
    for (int b = 0; b < bp.G; ++b) {
      if (b == blk) off = run;
      run = run + td.totals[b];
      if (b == blk) next = run;
    }
    s_off[0] = off;
    s_off[1] = next;
    s_off[2] = run;
  }
  __syncthreads();
  const double off = s_off[0], next = s_off[1], total = s_off[2];
  if (!(total > 0.0) || !isfinite(total)) {
    // f'' vanishes on the whole grid (or overflowed): uniform fallback.
    if (blk == 0) {
      for (int k = tid; k <= bp.N; k += kBuildThreads) write_uniform_knots(bp, td, k);
      if (tid == 0) *td.status = isfinite(total) ? PWL_FLAG_DEGENERATE : PWL_FLAG_NONFINITE;
    }
    return;
  }
  scan_block_cells(bp, blk, s_d, s_tp, s_S);
  const double dt = (bp.b - bp.a) / (double)bp.M;
  const double snap = 1e-12 * (bp.b - bp.a);
  for (int i = 1 + tid; i < bp.N; i += kBuildThreads) {
    const double tau = ((double)i * total) / (double)bp.N;
    if (!(off < tau && tau <= next)) continue;
    // smallest c with off + S_local[c] >= tau (exists: the last one equals next)
    int lo = 0, hi = C - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (off + s_S[mid] >= tau) hi = mid; else lo = mid + 1;
    }
    const double Sj = off + s_S[lo];
    const double Sp = (lo > 0) ? off + s_S[lo - 1] : off;
    const int j = blk * C + lo + 1;                    // 1-based cell number
    const double frac = (tau - Sp) / (Sj - Sp);
    double x = (bp.a + (double)(j - 1) * dt) + frac * dt;
    if (fabs(x) <= snap) x = 0.0;
    td.knots64[i] = x;
    td.knots[i] = (float)x;
  }
  if (blk == 0 && tid == 0) {
    td.knots64[0] = bp.a;
    td.knots[0] = (float)bp.a;
    td.knots64[bp.N] = bp.b;
    td.knots[bp.N] = (float)bp.b;
  }
}

__global__ __launch_bounds__(kBuildThreads) void k_segments(BuildParams bp, TableDev td) {
  const int k = blockIdx.x * kBuildThreads + threadIdx.x;
  if (k > bp.N) return;
  if (bp.partition == PWL_UNIFORM) {
    write_uniform_knots(bp, td, k);
  }
  float xk, xk1 = 0.0f;
  if (bp.partition == PWL_UNIFORM) {
#pragma clang fp contract(off)
    double x0 = bp.a + ((bp.b - bp.a) * (double)k) / (double)bp.N;
    if (k == 0) x0 = bp.a;
    if (k == bp.N) x0 = bp.b;
    xk = (float)x0;
    if (k < bp.N) {
      double x1 = bp.a + ((bp.b - bp.a) * (double)(k + 1)) / (double)bp.N;
      if (k + 1 == bp.N) x1 = bp.b;
      xk1 = (float)x1;
    }
  } else {
    xk = td.knots[k];
    if (k < bp.N) xk1 = td.knots[k + 1];
  }
  if (k >= 1 && k <= bp.N - 1) td.ucell[k] = map_cell(xk, bp.a32, bp.scale32, bp.K);
  if (bp.values == PWL_INTERP) {
    td.values[k] = f_value32(bp.f, xk);
  } else if (k < bp.N) {
    const float h = xk1 - xk;
    float sl = 0.0f, sr = 0.0f;
#pragma unroll
    for (int q = 0; q < kGaussPoints; ++q) {
      const float t = bp.gl.t[q];
      const float fq = bp.gl.w[q] * f_value32(bp.f, fmaf(h, t, xk));
      sl = fmaf(1.0f - t, fq, sl);
      sr = fmaf(t, fq, sr);
    }
    td.quad_l[k] = h * sl;
    td.quad_r[k] = h * sr;
  }
}

// Number of entries of the sorted array u[0..n) that are < key (lt) or <= key.
__device__ int count_below(const int32_t* u, int n, int key, bool inclusive) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool go_right = inclusive ? (u[mid] <= key) : (u[mid] < key);
    if (go_right) lo = mid + 1; else hi = mid;
  }
  return lo;
}

constexpr int kFinalizeThreads = 1024;
constexpr int kRowsPerThread = (PWL_MAX_N + 1 + kFinalizeThreads - 1) / kFinalizeThreads;

__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(BuildParams bp, TableDev td) {
  extern __shared__ double s_pcr[];
  const int N = bp.N, n = N + 1;
  const int tid = threadIdx.x;
  double* A = s_pcr;
  double* B = A + n;
  double* Cu = B + n;
  double* D = Cu + n;
  __shared__ int s_collapsed;
  if (tid == 0) s_collapsed = 0;
  __syncthreads();

  // 1. knot-collapse check on the FP32 knots
  int bad = 0;
  for (int k = tid; k < N; k += kFinalizeThreads)
    if (!(td.knots[k + 1] > td.knots[k])) bad = 1;
  if (bad) atomicOr(&s_collapsed, 1);
  __syncthreads();
  const bool collapsed = s_collapsed != 0;

  // 2. uniform index map: lo[u] = #{knots with cell < u}, count = #{cell == u}.
  // Strictly increasing knots have non-decreasing cells; a collapsed table
  // (evaluated as NaN) gets an empty map so no lookup leaves the table.
  // The largest count (knots sharing one cell) selects the evaluator's
  // unrolled compare depth.
  __shared__ int s_maxc;
  if (tid == 0) s_maxc = 0;
  __syncthreads();
  const int32_t* uc = td.ucell + 1;   // interior knots 1 .. N-1
  int my_max = 0;
  for (int u = tid; u < bp.K; u += kFinalizeThreads) {
    uint32_t e = 0u;
    if (!collapsed) {
      const int lo = count_below(uc, N - 1, u, false);
      const int hi = count_below(uc, N - 1, u, true);
      const int cnt = max(hi - lo, 0);
      e = (uint32_t)lo | ((uint32_t)cnt << 16);
      my_max = max(my_max, cnt);
    }
    td.cells[u] = e;
  }
  if (my_max > 0) atomicMax(&s_maxc, my_max);

  // 3. vertex values
  if (bp.values == PWL_PROJ) {
    // Gram matrix of the hat basis from the element matrix (h/6)[[2,1],[1,2]]
    // (half hats at both ends), right-hand side b_k = <f, phi_k>.
    for (int i = tid; i < n; i += kFinalizeThreads) {
      const double xi = (double)td.knots[i];
      const double hl = (i > 0) ? xi - (double)td.knots[i - 1] : 0.0;
      const double hr = (i < N) ? (double)td.knots[i + 1] - xi : 0.0;
      A[i] = hl / 6.0;
      Cu[i] = hr / 6.0;
      B[i] = hl / 3.0 + hr / 3.0;
      D[i] = ((i > 0) ? (double)td.quad_r[i - 1] : 0.0) + ((i < N) ? (double)td.quad_l[i] : 0.0);
    }
    __syncthreads();
    // Parallel cyclic reduction: at stride s every row eliminates its
    // couplings to rows i - s and i + s; after ceil(log2 n) steps the system
    // is diagonal.  No pivoting is needed: M is strictly diagonally dominant.
    for (int s = 1; s < n; s <<= 1) {
      double na[kRowsPerThread], nb[kRowsPerThread], nc[kRowsPerThread], nd[kRowsPerThread];
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int i = tid + r * kFinalizeThreads;
        if (i >= n) break;
        double ai = A[i], bi = B[i], ci = Cu[i], di = D[i];
        double an = 0.0, cn = 0.0;
        if (i - s >= 0) {
          const double al = -ai / B[i - s];
          an = al * A[i - s];
          bi += al * Cu[i - s];
          di += al * D[i - s];
        }
        if (i + s < n) {
          const double ga = -ci / B[i + s];
          cn = ga * Cu[i + s];
          bi += ga * A[i + s];
          di += ga * D[i + s];
        }
        na[r] = an; nb[r] = bi; nc[r] = cn; nd[r] = di;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int i = tid + r * kFinalizeThreads;
        if (i >= n) break;
        A[i] = na[r]; B[i] = nb[r]; Cu[i] = nc[r]; D[i] = nd[r];
      }
      __syncthreads();
    }
    for (int i = tid; i < n; i += kFinalizeThreads) D[i] = D[i] / B[i];
  } else {
    for (int i = tid; i < n; i += kFinalizeThreads) D[i] = (double)td.values[i];
  }
  __syncthreads();

  // 4. values, flags and packed records
  for (int i = tid; i < n; i += kFinalizeThreads) {
    const double c = D[i];
    td.values64[i] = c;
    td.values[i] = (float)c;
  }
  for (int k = tid; k < N; k += kFinalizeThreads) {
    const float x0 = td.knots[k], x1 = td.knots[k + 1];
    const double v0 = (double)(float)D[k], v1 = (double)(float)D[k + 1];
    const double h = (double)x1 - (double)x0;
    float4 r;
    r.x = x0;
    r.y = (float)D[k];
    r.z = (float)((v1 - v0) / h);
    r.w = (float)(1.0 / h);
    if (collapsed) {
      r.y = __builtin_nanf("");
      r.z = __builtin_nanf("");
    }
    td.rec[k] = r;
  }
  if (tid == 0) {
    uint32_t st = (bp.partition == PWL_UNIFORM) ? 0u : td.status[0];
    if (collapsed) st |= PWL_FLAG_KNOTS_COLLAPSED;
    td.status[0] = st;
    td.status[1] = (uint32_t)s_maxc;
  }
}

}  // namespace

hipError_t launch_build(const BuildParams& bp, const TableDev& td, hipStream_t s) {
  if (bp.partition == PWL_OPTIMAL) {
    hipLaunchKernelGGL(k_density_totals, dim3(bp.G), dim3(kBuildThreads), 0, s, bp, td);
    hipLaunchKernelGGL(k_invert_knots, dim3(bp.G), dim3(kBuildThreads), 0, s, bp, td);
  }
  const int nb = (bp.N + 1 + kBuildThreads - 1) / kBuildThreads;
  hipLaunchKernelGGL(k_segments, dim3(nb), dim3(kBuildThreads), 0, s, bp, td);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), finalize_lds_bytes(bp.N), s, bp, td);
  return hipGetLastError();
}

hipError_t configure_build_kernels(int max_lds) {
  const int want = (int)finalize_lds_bytes(PWL_MAX_N);
  return hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize,
                             want < max_lds ? want : max_lds);
}

}  // namespace pwl
