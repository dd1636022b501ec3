// Table construction on the GPU.
//
//   optimal partition (Sec. III-B1):
//     k_density_totals   FP64 |f''|^(2/5) on the fine grid, trapezoid sum per workgroup
//     k_invert_knots     FP64 prefix of those sums, targets i S_M / N, linear inversion;
//                        per knot also, for the interpolant, f(x_i)
//   every table:
//     k_finalize         one workgroup: uniform knots (Sec. IV) when asked, the
//                        uniform index map, the knot-collapse check, for the
//                        projection (Sec. II-B2) FP32 Gauss-Legendre integrals of f
//                        against the hats and the FP64 solve of M c = b (parallel
//                        cyclic reduction), and the packed records
//                        {x_k, v_k, slope_k, x_{k+1}}
#include <hip/hip_runtime.h>

#include "pwl_func.h"
#include "pwl_internal.h"
#include "pwl_locate.h"

namespace pwl {

namespace {

constexpr int kScanThreads = 1024;      // density workgroup size (one sample per thread)
constexpr int kScanLanes = 32;          // lanes that sum cells sequentially
constexpr int kCellsPerScanLane = kDensityCellsPerBlock / kScanLanes;   // 32

// Inclusive trapezoid sums of the density over the cells of workgroup `blk`.
// Cell j (1-based) spans [t_{j-1}, t_j], t_j = a + j dt, and adds
// (d_{j-1} + d_j) dt / 2.  All 1024 threads evaluate the density (one FP64
// sample each); then 32 lanes each sum 32 consecutive cells sequentially and
// lane 0 chains the 32 lane totals sequentially.  Every sum therefore
// extends the previous one by one rounded addition of a non-negative term,
// so the sums are monotone non-decreasing and the block total equals the
// last sum bit for bit; both kernels below call this same code.  Contraction
// is off so that every operation is one IEEE-rounded FP64 operation.
__device__ double scan_block_cells(const BuildParams& bp, int blk, double* s_d, double* s_tp,
                                   double* s_S) {
#pragma clang fp contract(off)
  constexpr int C = kDensityCellsPerBlock;
  const int tid = threadIdx.x;
  const double dt = (bp.b - bp.a) / (double)bp.M;
  const double hdt = dt / 2.0;
  const int j0 = blk * C;
  for (int s = tid; s <= C; s += kScanThreads) {
    const int j = j0 + s;
    s_d[s] = (j <= bp.M) ? knot_density(bp.f, bp.a + (double)j * dt) : 0.0;
  }
  __syncthreads();
  if (tid < kScanLanes) {
    double acc = 0.0;
#pragma unroll 8
    for (int q = 0; q < kCellsPerScanLane; ++q) {
      const int c = tid * kCellsPerScanLane + q;
      const double inc = (j0 + c + 1 <= bp.M) ? (s_d[c] + s_d[c + 1]) * hdt : 0.0;
      acc = acc + inc;
      if (s_S != nullptr) s_S[c] = acc;
    }
    s_tp[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double run = 0.0;
    for (int t = 0; t < kScanLanes; ++t) {
      const double v = s_tp[t];
      s_tp[t] = run;
      run = run + v;
    }
    s_tp[kScanLanes] = run;
  }
  __syncthreads();
  if (s_S != nullptr) {
    const int lane = tid / kCellsPerScanLane;   // 1024 threads cover the 1024 cells
    s_S[tid] = s_tp[lane] + s_S[tid];
  }
  const double total = s_tp[kScanLanes];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanThreads) void k_density_totals(BuildParams bp, TableDev td) {
  __shared__ double s_d[kDensityCellsPerBlock + 1];
  __shared__ double s_tp[kScanLanes + 1];
  const double tot = scan_block_cells(bp, blockIdx.x, s_d, s_tp, nullptr);
  if (threadIdx.x == 0) {
    td.totals[blockIdx.x] = tot;
    if (blockIdx.x == 0) {
      td.status[0] = 0u;
      td.status[1] = 0u;
    }
  }
}

__device__ double uniform_knot(const BuildParams& bp, int k) {
#pragma clang fp contract(off)
  double x = bp.a + ((bp.b - bp.a) * (double)k) / (double)bp.N;
  if (k == 0) x = bp.a;
  if (k == bp.N) x = bp.b;
  return x;
}

// Everything a knot needs once its position is known: FP64 and FP32 copies
// and, for the interpolant, f at the FP32 knot.
__device__ void emit_knot(const BuildParams& bp, const TableDev& td, int k, double x) {
  const float x32 = (float)x;
  td.knots64[k] = x;
  td.knots[k] = x32;
  if (bp.values == PWL_INTERP) td.values[k] = f_value32(bp.f, x32);
}

__global__ __launch_bounds__(kScanThreads) void k_invert_knots(BuildParams bp, TableDev td) {
#pragma clang fp contract(off)
  constexpr int C = kDensityCellsPerBlock;
  __shared__ double s_d[C + 1];
  __shared__ double s_S[C];
  __shared__ double s_tp[kScanLanes + 1];
  __shared__ double s_lane[kScanLanes + 1];
  __shared__ double s_tot[kMaxDensityBlocks];
  __shared__ double s_off[3];   // offset of this block, offset of the next, S_M
  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  for (int b = tid; b < bp.G; b += kScanThreads) s_tot[b] = td.totals[b];
  __syncthreads();
  // Prefix of the workgroup totals, chained in two sequential levels (32
  // lanes of consecutive totals, then the lane sums) so that the offset of
  // block b + 1 is, bit for bit, the offset of block b plus its total.
  const int per = (bp.G + kScanLanes - 1) / kScanLanes;
  const int my_lane = blk / per;
  if (tid < kScanLanes) {
    double acc = 0.0, before = 0.0, through = 0.0;
    for (int q = 0; q < per; ++q) {
      const int b = tid * per + q;
      if (b < bp.G) {
        if (b == blk) before = acc;
        acc = acc + s_tot[b];
        if (b == blk) through = acc;
      }
    }
    s_lane[tid] = acc;
    if (tid == my_lane) {
      s_off[0] = before;
      s_off[1] = through;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double run = 0.0, base = 0.0;
    for (int t = 0; t < kScanLanes; ++t) {
      if (t == my_lane) base = run;
      run = run + s_lane[t];
    }
    s_off[0] = base + s_off[0];
    s_off[1] = base + s_off[1];
    s_off[2] = run;
  }
  __syncthreads();
  const double off = s_off[0], next = s_off[1], total = s_off[2];
  if (!(total > 0.0) || !isfinite(total)) {
    // f'' vanishes on the whole grid (or overflowed): uniform fallback.
    if (blk == 0) {
      for (int k = tid; k <= bp.N; k += kScanThreads) emit_knot(bp, td, k, uniform_knot(bp, k));
      if (tid == 0) td.status[0] = isfinite(total) ? PWL_FLAG_DEGENERATE : PWL_FLAG_NONFINITE;
    }
    return;
  }
  scan_block_cells(bp, blk, s_d, s_tp, s_S);
  const double dt = (bp.b - bp.a) / (double)bp.M;
  const double snap = 1e-12 * (bp.b - bp.a);
  for (int i = 1 + tid; i < bp.N; i += kScanThreads) {
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
    emit_knot(bp, td, i, x);
  }
  if (blk == 0 && tid == 0) {
    emit_knot(bp, td, 0, bp.a);
    emit_knot(bp, td, bp.N, bp.b);
  }
}

constexpr int kFinalizeThreads = 1024;
constexpr int kRowsPerThread = (PWL_MAX_N + 1 + kFinalizeThreads - 1) / kFinalizeThreads;

// Everything after the knots, in one workgroup that keeps the knots and their
// map cells in LDS (every later step reads them several times):
//  1. (uniform partition) the knots x_k = a + (b - a) k / N and their
//     interpolant values; otherwise the knots the inversion wrote;
//  2. per segment k: its cells of the uniform index map lo[u] = #{interior
//     knots with cell < u} - segment k owns (cell(x_k), cell(x_{k+1})], with
//     cell(x_0) = -1 and cell(x_N) = K - 1, so each cell is written once when
//     the knots increase; the knot-collapse check; the deepest cell (the
//     evaluator's unrolled compare depth);
//  3. (projection) <f, phi_k> by 16-point Gauss-Legendre per segment, one
//     thread per segment;
//  4. (projection) the FP64 solve of M c = b by parallel cyclic reduction;
//  5. the packed records {x_k, v_k, slope_k, x_{k+1}} (NaN for a collapsed
//     table, whose map is then cleared).
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(BuildParams bp, TableDev td) {
  extern __shared__ double s_pcr[];
  const int N = bp.N, n = N + 1;
  const int tid = threadIdx.x;
  double* A = s_pcr;
  double* R = A + n;      // reciprocal diagonal during the solve
  double* Cu = R + n;
  double* D = Cu + n;
  float* X = reinterpret_cast<float*>(D + n);        // [N+1] FP32 knots
  uint16_t* U = reinterpret_cast<uint16_t*>(X + n);  // [N+1] map cell of each interior knot
  __shared__ int s_collapsed, s_maxc;
  if (tid == 0) {
    s_collapsed = 0;
    s_maxc = 0;
  }
  // 1. knots (and, for the uniform interpolant, the values) into LDS
  const bool uniform = bp.partition == PWL_UNIFORM;
  for (int k = tid; k <= N; k += kFinalizeThreads) {
    float x32;
    if (uniform) {
      const double x = uniform_knot(bp, k);
      x32 = (float)x;
      td.knots64[k] = x;
      td.knots[k] = x32;
      if (bp.values == PWL_INTERP) D[k] = (double)f_value32(bp.f, x32);
    } else {
      x32 = td.knots[k];
      if (bp.values == PWL_INTERP) D[k] = (double)td.values[k];
    }
    X[k] = x32;
    U[k] = (k >= 1 && k <= N - 1) ? (uint16_t)map_cell(x32, bp.a32, bp.scale32, bp.K) : (uint16_t)0;
  }
  __syncthreads();

  // 2. map, collapse check, deepest cell
  int run = 0, bad = 0;
  for (int k = tid; k < N; k += kFinalizeThreads) {
    const int u0 = (k == 0) ? -1 : (int)U[k];
    const int u1 = (k + 1 == N) ? bp.K - 1 : (int)U[k + 1];
    for (int u = u0 + 1; u <= u1; ++u) td.lo[u] = (uint16_t)k;
    if (!(X[k + 1] > X[k])) bad = 1;
    if (k >= 1 && (k == 1 || (int)U[k - 1] != u0)) {   // first interior knot of its cell
      int r = 1;
      while (k + r <= N - 1 && (int)U[k + r] == u0) ++r;
      run = max(run, r);
    }
  }
  if (tid == 0) td.lo[bp.K] = (uint16_t)(N - 1);
  if (bad) atomicOr(&s_collapsed, 1);
  if (run > 0) atomicMax(&s_maxc, run);

  // 3-4. vertex values
  if (bp.values == PWL_PROJ) {
    // one thread per segment k: its 16 Gauss-Legendre nodes in order;
    // L_k = <f, phi_k> on segment k goes to D[k], R_k = <f, phi_{k+1}> to A[k+1]
    for (int k = tid; k < N; k += kFinalizeThreads) {
      const float xk = X[k];
      const float h = X[k + 1] - xk;
      float sl = 0.0f, sr = 0.0f;
#pragma unroll
      for (int q = 0; q < kGaussPoints; ++q) {
        const float t = bp.gl.t[q];
        const float fq = bp.gl.w[q] * f_value32(bp.f, fmaf(h, t, xk));
        sl = fmaf(1.0f - t, fq, sl);
        sr = fmaf(t, fq, sr);
      }
      D[k] = (double)(h * sl);
      A[k + 1] = (double)(h * sr);
    }
    __syncthreads();
    // Gram matrix of the hat basis from the element matrix (h/6)[[2,1],[1,2]]
    // (half hats at both ends), right-hand side b_k = <f, phi_k>.  Row i is
    // owned by thread i mod 1024 for the whole solve: it keeps its diagonal
    // in registers and publishes the reciprocal for its neighbours.
    double diag[kRowsPerThread];
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
      const int i = tid + r * kFinalizeThreads;
      if (i >= n) break;
      const double xi = (double)X[i];
      const double hl = (i > 0) ? xi - (double)X[i - 1] : 0.0;
      const double hr = (i < N) ? (double)X[i + 1] - xi : 0.0;
      const double bl = (i > 0) ? A[i] : 0.0;
      const double br = (i < N) ? D[i] : 0.0;
      D[i] = bl + br;
      A[i] = hl / 6.0;
      Cu[i] = hr / 6.0;
      diag[r] = hl / 3.0 + hr / 3.0;
      R[i] = 1.0 / diag[r];
    }
    __syncthreads();
    // Parallel cyclic reduction: at stride s every row eliminates its
    // couplings to rows i - s and i + s; after ceil(log2 n) steps the system
    // is diagonal.  No pivoting is needed: M is strictly diagonally dominant.
    for (int s = 1; s < n; s <<= 1) {
      double na[kRowsPerThread], nc[kRowsPerThread], nd[kRowsPerThread];
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int i = tid + r * kFinalizeThreads;
        if (i >= n) break;
        double bi = diag[r], di = D[i];
        double an = 0.0, cn = 0.0;
        if (i - s >= 0) {
          const double al = -A[i] * R[i - s];
          an = al * A[i - s];
          bi += al * Cu[i - s];
          di += al * D[i - s];
        }
        if (i + s < n) {
          const double ga = -Cu[i] * R[i + s];
          cn = ga * Cu[i + s];
          bi += ga * A[i + s];
          di += ga * D[i + s];
        }
        na[r] = an; diag[r] = bi; nc[r] = cn; nd[r] = di;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int i = tid + r * kFinalizeThreads;
        if (i >= n) break;
        A[i] = na[r]; Cu[i] = nc[r]; D[i] = nd[r];
        R[i] = 1.0 / diag[r];
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
      const int i = tid + r * kFinalizeThreads;
      if (i >= n) break;
      D[i] = D[i] / diag[r];
    }
  }
  __syncthreads();

  // 5. values, flags and packed records
  const bool collapsed = s_collapsed != 0;
  if (collapsed)   // the evaluators never leave the table through an all-zero map
    for (int u = tid; u < bp.K; u += kFinalizeThreads) td.lo[u] = 0;
  for (int i = tid; i < n; i += kFinalizeThreads) {
    const double c = D[i];
    td.values64[i] = c;
    td.values[i] = (float)c;
  }
  for (int k = tid; k < N; k += kFinalizeThreads) {
    const float x0 = X[k], x1 = X[k + 1];
    const double v0 = (double)(float)D[k], v1 = (double)(float)D[k + 1];
    const double h = (double)x1 - (double)x0;
    float4 r;
    r.x = x0;
    r.y = (float)D[k];
    r.z = (float)((v1 - v0) / h);
    r.w = x1;
    if (collapsed) {
      r.y = __builtin_nanf("");
      r.z = __builtin_nanf("");
    }
    td.rec[k] = r;
  }
  if (tid == 0) {
    // the density kernels may have raised DEGENERATE / NONFINITE
    uint32_t st = (bp.partition == PWL_OPTIMAL) ? td.status[0] : 0u;
    if (collapsed) st |= PWL_FLAG_KNOTS_COLLAPSED;
    td.status[0] = st;
    td.status[1] = (uint32_t)s_maxc;
  }
}

// ---- error-prediction integrals (choice of N for a target error) ----------
constexpr int kNormThreads = 1024;

// Block b of the fine grid t_j = a + j (b - a) / Q, j = 0..Q: trapezoid
// weights times |f''|^(2/5) and f''^2, and max |f''|, reduced in FP64 in a
// fixed order (a tree over the block's threads).
__global__ __launch_bounds__(kNormThreads) void k_norms(FuncDesc f, double a, double b, int Q,
                                                        double* __restrict__ part) {
  __shared__ double s_d[kNormThreads], s_q[kNormThreads], s_m[kNormThreads];
  const int tid = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * kNormThreads + tid;
  const double dt = (b - a) / (double)Q;
  double d = 0.0, q = 0.0, m = 0.0;
  if (j <= Q) {
    const double x = a + (double)j * dt;
    const double f2 = f_second64(f, x);
    const double w = (j == 0 || j == Q) ? 0.5 * dt : dt;
    d = w * knot_density(f, x);
    q = w * f2 * f2;
    m = fabs(f2);
  }
  s_d[tid] = d;
  s_q[tid] = q;
  s_m[tid] = m;
  __syncthreads();
  for (int h = kNormThreads / 2; h >= 1; h >>= 1) {
    if (tid < h) {
      s_d[tid] += s_d[tid + h];
      s_q[tid] += s_q[tid + h];
      s_m[tid] = fmax(s_m[tid], s_m[tid + h]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[3 * blockIdx.x] = s_d[0];
    part[3 * blockIdx.x + 1] = s_q[0];
    part[3 * blockIdx.x + 2] = s_m[0];
  }
}

// One thread adds the G block results in order: out = {int |f''|^(2/5),
// int f''^2, max |f''|}.
__global__ void k_norms_final(const double* __restrict__ part, int G, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double d = 0.0, q = 0.0, m = 0.0;
  for (int g = 0; g < G; ++g) {
    d += part[3 * g];
    q += part[3 * g + 1];
    m = fmax(m, part[3 * g + 2]);
  }
  out[0] = d;
  out[1] = q;
  out[2] = m;
}

}  // namespace

int norm_blocks(int Q) { return Q / kNormThreads + 1; }

hipError_t launch_norms(const FuncDesc& f, double a, double b, int Q, double* scratch, hipStream_t s) {
  const int G = norm_blocks(Q);
  hipLaunchKernelGGL(k_norms, dim3(G), dim3(kNormThreads), 0, s, f, a, b, Q, scratch);
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(64), 0, s, scratch, G, scratch + 3 * G);
  return hipGetLastError();
}

hipError_t launch_build(const BuildParams& bp, const TableDev& td, hipStream_t s) {
  if (bp.partition == PWL_OPTIMAL) {
    hipLaunchKernelGGL(k_density_totals, dim3(bp.G), dim3(kScanThreads), 0, s, bp, td);
    hipLaunchKernelGGL(k_invert_knots, dim3(bp.G), dim3(kScanThreads), 0, s, bp, td);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), finalize_lds_bytes(bp.N), s, bp, td);
  return hipGetLastError();
}

hipError_t configure_build_kernels(int max_lds) {
  const int want = (int)finalize_lds_bytes(PWL_MAX_N);
  return hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize,
                             want < max_lds ? want : max_lds);
}

}  // namespace pwl
