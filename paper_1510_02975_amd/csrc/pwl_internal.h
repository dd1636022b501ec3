// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "pwl.h"

namespace pwl {

constexpr int kFineCellsPerSegment = 256;   // M = 256 N density cells
constexpr int kDensityCellsPerBlock = 1024; // cells scanned by one build workgroup
constexpr int kMaxDensityBlocks = kFineCellsPerSegment * PWL_MAX_N / kDensityCellsPerBlock;
constexpr int kBuildThreads = 256;
constexpr int kGaussPoints = 16;            // Gauss-Legendre nodes per segment for <f, phi_k>
constexpr int kKnotPad = 8;                 // NaN sentinels after the last interior knot in LDS
constexpr int kMaxUnrolledCount = 4;        // knots per map cell handled by unrolled compares

// The function f and its parameters, resolved on the host (defaults filled in).
struct FuncDesc {
  int32_t func;
  int32_t nparams;
  double p[PWL_MAX_PARAMS];   // Gaussian {s, amp}; Lorentzian {g, amp}; J0 {amp}; poly c0..c5; exp {alpha, amp}
  float p32[PWL_MAX_PARAMS];  // the same, rounded to FP32 (FP32 evaluations)
  // PWL_F_SAMPLED: f and f'' at t_i = s_a + i s_h, i = 0..S (device FP64)
  const double* sf;
  const double* sf2;
  int32_t S;
  double s_a, s_h;
};

// Device view of a table's persistent arrays.
struct TableDev {
  float4* rec;        // [N]   {x_k, v_k, slope_k, x_{k+1}}
  float* knots;       // [N+1] FP32 knots
  uint16_t* lo;       // [K+1] uniform index map: lo[u] = #{interior knots in cells < u}
  float* values;      // [N+1] FP32 vertex values
  double* knots64;    // [N+1] FP64 knots before rounding
  double* values64;   // [N+1] FP64 vertex values
  uint32_t* status;   // [0] build flags (PWL_FLAG_*), [1] most knots in one map cell
  // build scratch
  double* totals;     // [G] per-workgroup density sums
};

// Everything an evaluation kernel needs about a table.
struct EvalTable {
  const float4* rec;
  const float* knots;
  const uint16_t* lo;        // [K+1] uniform index map
  const uint32_t* meta;      // [0] build flags, [1] most knots sharing one map cell
  int32_t N, K;
  float a32, b32, scale32;   // cell(x) = floor((x - a32) * scale32), clamped to [0, K-1]
};

// Gauss-Legendre rule on [0, 1].
struct GaussRule {
  float t[kGaussPoints];
  float w[kGaussPoints];
};

struct BuildParams {
  FuncDesc f;
  double a, b;       // FP32-rounded domain, promoted
  float a32, b32, scale32;
  int32_t N, K, M, G;
  int32_t partition, values;
  GaussRule gl;
};

// The LDS image of a table, in 16-byte words, each section starting on a
// word: the N records, the knots with their NaN sentinels (N + kKnotPad
// floats) and the u16 map lo[0..K], the last two rounded up to whole words.
__host__ __device__ inline int image_knot_words(int N) { return (N + kKnotPad + 3) / 4; }
__host__ __device__ inline int image_map_words(int K) { return (K + 1 + 7) / 8; }
__host__ __device__ inline int image_words(int N, int K) { return N + image_knot_words(N) + image_map_words(K); }
// The structure-of-arrays variant (forward only): each of the four record
// fields is an array of N floats rounded up to whole words.
__host__ __device__ inline int image_soa_field_words(int N) { return (N + 3) / 4; }
__host__ __device__ inline int image_words_soa(int N, int K) {
  return 4 * image_soa_field_words(N) + image_knot_words(N) + image_map_words(K);
}

// Copies of a workgroup's FP64 dL/dv in LDS (backward kernels): lane l adds
// into copy l mod copies.  With few entries the 64 lanes of a wave would
// otherwise often add into the same entry, and same-address LDS atomics of
// one instruction serialise; the copies are summed, in order, at the flush.
__host__ __device__ inline int dv_copies(int N) {
  const int m = N + 1;   // at most 1024 doubles (8 KB) in all
  return m <= 64 ? 16 : (m <= 128 ? 8 : (m <= 256 ? 4 : (m <= 512 ? 2 : 1)));
}

// LDS bytes of the evaluation kernels for a table of N segments and K cells:
// the image, then (backward) the workgroup's FP64 dL/dv.
inline size_t eval_lds_bytes(int N, int K, bool backward) {
  size_t b = 16 * (size_t)image_words(N, K);
  if (backward) b += sizeof(double) * (size_t)(N + 1) * (size_t)dv_copies(N);
  return b;
}

inline size_t eval_lds_bytes_soa(int N, int K) { return 16 * (size_t)image_words_soa(N, K); }
// The value/slope-pairs variant (forward only): two 8-byte pairs per word.
__host__ __device__ inline int image_pair_words(int N) { return (N + 1) / 2; }
inline size_t eval_lds_bytes_pairs(int N, int K) {
  return 16 * (size_t)(image_pair_words(N) + image_knot_words(N) + image_map_words(K));
}

// Table finalize: 4 FP64 PCR rows, the FP32 knots and their u16 map cells.
inline size_t finalize_lds_bytes(int N) {
  return (4 * sizeof(double) + sizeof(float) + sizeof(uint16_t)) * (size_t)(N + 1);
}

// Number of map cells for a table of N segments: two per segment on a uniform
// partition (each cell then holds at most one knot), four on the optimal one.
// Index-map cells: 2N for a uniform partition, 4N for the optimal one or 8N
// where its knots crowd (chosen per table when it is built; N at most
// kWideMapMaxN).  The allocation holds the largest map an N can get.
constexpr int kWideMapMaxN = 2048;
inline int map_cells_max(int N) { return N <= kWideMapMaxN ? 8 * N : 4 * N; }

struct LaunchShape {
  int block;
  int grid;
  size_t lds;
};

// Tunable launch configuration of a streaming kernel family.
struct LaunchConfig {
  int unroll;      // float4 vectors per thread per iteration (1, 2 or 4)
  int block;       // threads per workgroup (multiple of 64, <= 1024)
  int wg_per_cu;   // workgroups per CU (capped by the table's LDS footprint)
};

hipError_t set_launch(int kernel, int unroll, int block, int wg_per_cu);
LaunchConfig get_launch(int kernel);
hipError_t set_locate(int mode);
int get_locate();
hipError_t set_records(int layout);
int get_records();

// ---- batched evaluation ----------------------------------------------------
// A batch copies every table's LDS image (the layout carve() describes:
// records, NaN-padded knots, index map) into one arena at creation, in table
// order.  A workgroup copies the images of all the tables its runs touch -
// one contiguous span of the arena - into LDS once, then streams its runs
// without further barriers.
struct BatchTable {          // one table of a batch, for packing its image
  EvalTable t;               // the table's own arrays and shape
  float4* img;               // its LDS image in the batch arena
  int32_t nvec;              // image size in 16-byte words
  int32_t pad;
};

// Points [begin, end) of one table, handled by one workgroup, with the
// table's shape copied in: a workgroup reads nothing else to evaluate it.
struct BatchRun {
  int32_t img_lds;           // the table's image: 16-byte word offset in the workgroup's LDS
  int32_t dv_lds;            // backward: word offset of the table's FP64 dL/dv in LDS
  int64_t begin, end;
  int64_t part;              // backward: first of the run's N + 1 partial dL/dv sums in the batch's buffer
  int32_t table, nvec, N, K;
  float a32, b32, scale32;
  int32_t maxc;              // most knots sharing one map cell (the unrolled compare depth)
};
static_assert(sizeof(BatchRun) == 64, "BatchRun is 64 bytes");

// One work unit of a batched launch: runs [r0, r1) and the arena words
// [img, img + nwords) holding their tables' images; the backward's dL/dv
// regions follow the images in LDS (dv_words 16-byte words from word
// dv_lds).  maxc: the deepest map cell among its runs' tables.
struct BatchGroup {
  int64_t img;
  int32_t nwords;
  int32_t r0, r1;
  int32_t dv_lds, dv_words;
  int32_t maxc;
};
static_assert(sizeof(BatchGroup) == 32, "BatchGroup is 32 bytes");

// LDS of one table in a batched workgroup: its image and (backward) its FP64
// dL/dv, in 16-byte words.
inline int batch_dv_words(int N) { return ((N + 1) * dv_copies(N) * (int)sizeof(double) + 15) / 16; }
inline size_t batch_table_lds_bytes(int N, int K, bool backward) {
  return 16 * ((size_t)image_words(N, K) + (backward ? (size_t)batch_dv_words(N) : 0));
}

struct BatchPlan {           // the work units of one launch
  BatchRun* runs;            // device
  BatchGroup* groups;        // device [ngroups]
  const float4* arena;       // device: the images, table 0 first
  int32_t grid;              // workgroups launched (the forward's take groups grid apart, the backward's one each)
  int32_t ngroups;
  int32_t nruns;
  size_t lds;                // the largest group's LDS bytes
};

// One launch per direction over all the tables.
struct BatchLaunch {
  BatchPlan fwd, bwd;
  int64_t dv_len;            // sum over tables of N + 1
  int32_t T;
  int32_t max_n;             // the largest table's N
  float* part;               // device: every backward run's N + 1 partial dL/dv sums
  const int64_t* tab_part;   // device: per table, in table order, its runs' offsets into part in slice order
  const int32_t* tab_first;  // device [T + 1]: table t's entries of tab_part are [tab_first[t], tab_first[t+1])
  const int64_t* tab_dv;     // device [T + 1]: table t's gradients are dv[tab_dv[t] .. tab_dv[t+1])
};

hipError_t launch_batch(const BatchLaunch& bl, const float* x, const float* g, float* y, float* dx,
                        float* dv, hipStream_t s);
// Writes every table's image and its deepest map cell (maxc[T]).
hipError_t launch_batch_pack(const BatchTable* tabs, int T, int32_t* maxc, hipStream_t s);
hipError_t configure_batch_kernels(int max_lds);

// ---- launchers (defined in the .hip files) --------------------------------
hipError_t launch_build(const BuildParams& bp, const TableDev& td, hipStream_t s);
// The integrals behind the error predictions, on Q trapezoid cells of [a, b]:
// scratch holds 3 * norm_blocks(Q) partial sums, then {int |f''|^(2/5),
// int f''^2, max |f''|}.
int norm_blocks(int Q);
hipError_t launch_norms(const FuncDesc& f, double a, double b, int Q, double* scratch, hipStream_t s);
hipError_t launch_eval(const EvalTable& t, const float* v_override, const float* x, float* y,
                       int64_t n, int num_cu, hipStream_t s);
// The fused backward writes one row of dL/dv partial sums per workgroup into
// `part` and adds the rows in a second kernel; the rows it needs:
size_t backward_workspace_floats(const EvalTable& t, const float* x, const float* g, const float* y,
                                 const float* dx, int64_t n, int num_cu);
hipError_t launch_eval_backward(const EvalTable& t, const float* v_override, const float* x,
                                const float* g, float* y, float* dx, float* dv, float* part, int64_t n,
                                int num_cu, hipStream_t s);
hipError_t launch_locate(const EvalTable& t, const float* x, int32_t* seg, int64_t n, int num_cu,
                         hipStream_t s);
hipError_t launch_direct_gaussian(const float* x, float* y, int64_t n, float s, float amp, int fast,
                                  int num_cu, hipStream_t st);
hipError_t launch_copy(const float* src, float* dst, int64_t n, int num_cu, hipStream_t s);
hipError_t launch_direct_func(const FuncDesc& f, const float* x, float* y, int64_t n, int num_cu, hipStream_t s);
hipError_t launch_kde(const EvalTable& t, int mode, const void* frame, const void* hist, int H, int W, int T,
                      int r, const float* sigma, float* out, hipStream_t s);
hipError_t configure_kde_kernels(int max_lds);
hipError_t configure_kernels();   // raise dynamic-LDS limits once per process

}  // namespace pwl
