// Host runtime behind the C ABI declared in include/pwl.h: argument
// validation (pure host, before any HIP call), the per-table device arena,
// launch of the build pipeline and of the evaluation kernels, and error
// reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pwl.h"
#include "pwl_internal.h"

namespace pwl {
hipError_t configure_build_kernels(int max_lds);
hipError_t configure_kde_kernels(int max_lds);
hipError_t configure_eval_kernels(int max_lds);
}  // namespace pwl

struct pwl_batch {
  int device;
  int32_t T;
  int64_t npoints;
  pwl::BatchLaunch bl;
  void* base;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct pwl_table {
  int device;
  int kcap;   // map cells the arena can hold
  pwl::BuildParams bp;
  pwl::TableDev td;
  void* base;
  size_t bytes;
  hipEvent_t built = nullptr;   // recorded after every build of the table
  // dL/dv partial sums of the fused backward (one row per workgroup), taken
  // from the stream-ordered allocator by the first backward call that needs
  // more; part_used is recorded after every launch that reads them
  mutable std::mutex part_mu;
  mutable float* part = nullptr;
  mutable size_t part_cap = 0;   // floats
  mutable hipEvent_t part_used = nullptr;
};

namespace {

thread_local std::string g_err;

pwl_status fail(pwl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define PWL_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(PWL_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
  } while (0)

// ---- device properties and one-time kernel configuration -------------------

constexpr int kMaxDevices = 64;
// Device scratch of pwl_eval_backward_noalloc: the fused backward's dL/dv
// partial sums (one row of N + 1 per workgroup), at most kScratchFloats
// floats (8 MiB).  Every device that runs the library holds its own copy
// until the process ends.  Host code reaches it only through the device
// address taken once per device at set-up (g_scratch): the array's name is a
// host-side stand-in, not a device address.
constexpr size_t kScratchFloats = size_t(1) << 21;
static __device__ __align__(256) float scratch[kScratchFloats];

int g_num_cu[kMaxDevices];
int g_max_lds[kMaxDevices];
float* g_scratch[kMaxDevices];   // this device's `scratch`
hipStream_t g_aux[kMaxDevices];   // library-internal stream for small host reads
std::once_flag g_cfg_once[kMaxDevices];
hipError_t g_cfg_err[kMaxDevices];

pwl_status device_ready(int* dev_out, int* num_cu, int* max_lds = nullptr) {
  int dev = 0;
  PWL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PWL_EHIP, "device ordinal %d out of range", dev);
  std::call_once(g_cfg_once[dev], [dev]() {
    int cu = 0, lds = 0;
    hipError_t e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = pwl::configure_build_kernels(lds);
    if (e == hipSuccess) e = pwl::configure_eval_kernels(lds);
    if (e == hipSuccess) e = pwl::configure_batch_kernels(lds);
    if (e == hipSuccess) e = pwl::configure_kde_kernels(lds);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g_aux[dev], hipStreamNonBlocking);
    void* sp = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    g_scratch[dev] = static_cast<float*>(sp);
    g_num_cu[dev] = cu > 0 ? cu : 1;
    g_max_lds[dev] = lds;
    g_cfg_err[dev] = e;
  });
  if (g_cfg_err[dev] != hipSuccess)
    return fail(PWL_EHIP, "kernel configuration failed: %s", hipGetErrorString(g_cfg_err[dev]));
  if (dev_out) *dev_out = dev;
  if (num_cu) *num_cu = g_num_cu[dev];
  if (max_lds) *max_lds = g_max_lds[dev];
  return PWL_OK;
}

// ---- Gauss-Legendre rule on [0, 1] (Newton on the Legendre recurrence) ------

pwl::GaussRule make_gauss_rule() {
  const int n = pwl::kGaussPoints;
  pwl::GaussRule r;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double w = 2.0 / ((1.0 - z * z) * dp * dp);
    r.t[i] = (float)((1.0 - z) / 2.0);   // map [-1, 1] -> [0, 1]
    r.w[i] = (float)(w / 2.0);
  }
  return r;
}

const pwl::GaussRule& gauss_rule() {
  static const pwl::GaussRule r = make_gauss_rule();
  return r;
}

// ---- argument resolution ----------------------------------------------------

pwl_status resolve_func(int32_t func, const double* params, int32_t nparams, pwl::FuncDesc* fd) {
  if (nparams < 0 || nparams > PWL_MAX_PARAMS)
    return fail(PWL_EINVAL, "nparams must be in [0, %d], got %d", PWL_MAX_PARAMS, nparams);
  if (nparams > 0 && params == nullptr) return fail(PWL_EINVAL, "params is NULL but nparams = %d", nparams);
  for (int i = 0; i < nparams; ++i)
    if (!std::isfinite(params[i])) return fail(PWL_EINVAL, "params[%d] is not finite", i);
  std::memset(fd, 0, sizeof(*fd));
  fd->func = func;
  fd->nparams = nparams;
  auto get = [&](int i, double def) { return i < nparams ? params[i] : def; };
  switch (func) {
    case PWL_F_GAUSSIAN:
    case PWL_F_LORENTZIAN:
      if (nparams > 2) return fail(PWL_EINVAL, "this function takes at most 2 parameters");
      fd->p[0] = get(0, 1.0);
      fd->p[1] = get(1, 1.0);
      if (!(fd->p[0] > 0.0)) return fail(PWL_EINVAL, "width parameter must be > 0");
      break;
    case PWL_F_BESSEL_J0:
      if (nparams > 1) return fail(PWL_EINVAL, "J0 takes at most 1 parameter (amp)");
      fd->p[0] = get(0, 1.0);
      break;
    case PWL_F_POLY:
      for (int i = 0; i < PWL_MAX_PARAMS; ++i) fd->p[i] = get(i, 0.0);
      break;
    case PWL_F_SAMPLED:
      return fail(PWL_EINVAL, "a sampled function is built with pwl_build_sampled");
    case PWL_F_EXP:
      if (nparams > 2) return fail(PWL_EINVAL, "exp takes at most 2 parameters");
      fd->p[0] = get(0, 1.0);
      fd->p[1] = get(1, 1.0);
      break;
    default:
      return fail(PWL_EINVAL, "unknown function id %d", func);
  }
  for (int i = 0; i < PWL_MAX_PARAMS; ++i) fd->p32[i] = (float)fd->p[i];
  return PWL_OK;
}

// f'' on the host, only to size the index map (the device evaluates its
// own); NaN for sampled functions, whose samples live on the device.
double host_second(const pwl::FuncDesc& f, double x) {
  switch (f.func) {
    case PWL_F_GAUSSIAN: {
      const double s2 = f.p[0] * f.p[0];
      return f.p[1] * ((x * x) / (s2 * s2) - 1.0 / s2) * std::exp(-(x * x) / (2.0 * s2));
    }
    case PWL_F_LORENTZIAN: {
      const double u = x / f.p[0], q = 1.0 + u * u;
      return f.p[1] * (6.0 * u * u - 2.0) / (f.p[0] * f.p[0] * q * q * q);
    }
    case PWL_F_BESSEL_J0:
      return (x == 0.0) ? -0.5 * f.p[0] : f.p[0] * (::j1(x) / x - ::j0(x));
    case PWL_F_POLY: {
      double r = 0.0;
      for (int k = PWL_MAX_PARAMS - 1; k >= 2; --k) r = r * x + (double)(k * (k - 1)) * f.p[k];
      return r;
    }
    case PWL_F_EXP:
      return f.p[1] * f.p[0] * f.p[0] * std::exp(f.p[0] * x);
    default:
      return std::nan("");
  }
}

// Map cells of a table.  The optimal partition puts about N rho(x)(b - a)/K
// knots in the cell at x, rho the normalised density |f''|^(2/5); where that
// exceeds 1.5 at K = 4N some cell holds three knots and every point pays a
// third compare, so the map doubles to 8N cells (at most two knots a cell,
// which cost the evaluator one paired read like one).  The density is
// sampled at 512 points; the choice changes only the evaluators' speed,
// never a result, because the map is exact for any K.
int choose_map_cells(const pwl::BuildParams& bp, int partition) {
  const int N = bp.N;
  if (partition == PWL_UNIFORM) return 2 * N;
  if (N > pwl::kWideMapMaxN) return 4 * N;
  constexpr int kSamples = 512;
  double sum = 0.0, peak = 0.0;
  for (int i = 0; i < kSamples; ++i) {
    const double x = bp.a + (bp.b - bp.a) * ((double)i + 0.5) / kSamples;
    const double d = std::pow(std::fabs(host_second(bp.f, x)), 0.4);
    if (!std::isfinite(d)) return 4 * N;
    sum += d;
    peak = std::max(peak, d);
  }
  if (!(sum > 0.0)) return 4 * N;
  return (peak / (4.0 * (sum / kSamples)) > 1.5) ? 8 * N : 4 * N;
}

pwl_status resolve_build(int32_t func, const double* params, int32_t nparams, double a, double b,
                         int32_t N, int32_t partition, int32_t values, pwl::BuildParams* bp) {
  if (N < 1) return fail(PWL_EINVAL, "N must be >= 1, got %d", N);
  if (N > PWL_MAX_N) return fail(PWL_ECAPACITY, "N = %d exceeds PWL_MAX_N = %d", N, PWL_MAX_N);
  if (partition != PWL_UNIFORM && partition != PWL_OPTIMAL)
    return fail(PWL_EINVAL, "unknown partition %d", partition);
  if (values != PWL_INTERP && values != PWL_PROJ) return fail(PWL_EINVAL, "unknown values kind %d", values);
  if (!std::isfinite(a) || !std::isfinite(b)) return fail(PWL_EINVAL, "a and b must be finite");
  const float a32 = (float)a, b32 = (float)b;
  if (!std::isfinite(a32) || !std::isfinite(b32) || !(a32 < b32))
    return fail(PWL_EINVAL, "need a < b after rounding to FP32 (a=%g, b=%g)", a, b);
  std::memset(bp, 0, sizeof(*bp));
  pwl_status st = resolve_func(func, params, nparams, &bp->f);
  if (st != PWL_OK) return st;
  bp->a = (double)a32;
  bp->b = (double)b32;
  bp->a32 = a32;
  bp->b32 = b32;
  bp->N = N;
  bp->K = choose_map_cells(*bp, partition);
  bp->scale32 = (float)((double)bp->K / (bp->b - bp->a));
  bp->M = pwl::kFineCellsPerSegment * N;
  bp->G = (bp->M + pwl::kDensityCellsPerBlock - 1) / pwl::kDensityCellsPerBlock;
  bp->partition = partition;
  bp->values = values;
  bp->gl = gauss_rule();
  if (!std::isfinite(bp->scale32) || !(bp->scale32 > 0.0f))
    return fail(PWL_EINVAL, "domain too narrow for the index map");
  return PWL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves the table's arrays out of one allocation (base may be null to size it).
size_t layout(pwl::TableDev* td, char* base, int N, int K, int G) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  td->rec = reinterpret_cast<float4*>(take(sizeof(float4) * N));
  td->knots = reinterpret_cast<float*>(take(sizeof(float) * (N + 1)));
  td->lo = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * (K + 1)));
  td->values = reinterpret_cast<float*>(take(sizeof(float) * (N + 1)));
  td->knots64 = reinterpret_cast<double*>(take(sizeof(double) * (N + 1)));
  td->values64 = reinterpret_cast<double*>(take(sizeof(double) * (N + 1)));
  td->status = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 4));
  td->totals = reinterpret_cast<double*>(take(sizeof(double) * G));
  return off;
}

pwl::EvalTable eval_view(const pwl_table* t) {
  pwl::EvalTable e;
  e.rec = t->td.rec;
  e.knots = t->td.knots;
  e.lo = t->td.lo;
  e.meta = t->td.status;
  e.N = t->bp.N;
  e.K = t->bp.K;
  e.a32 = t->bp.a32;
  e.b32 = t->bp.b32;
  e.scale32 = t->bp.scale32;
  return e;
}

pwl_status check_table(const pwl_table* t, int* num_cu) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  int dev = 0;
  pwl_status st = device_ready(&dev, num_cu);
  if (st != PWL_OK) return st;
  if (dev != t->device)
    return fail(PWL_EINVAL, "table lives on device %d but device %d is current", t->device, dev);
  return PWL_OK;
}

}  // namespace

extern "C" {

int32_t pwl_abi_version(void) { return PWL_ABI_VERSION; }

const char* pwl_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Allocates a table for resolved build parameters and enqueues its build.
pwl_status create_table(const pwl::BuildParams& bp, void* stream, pwl_table** out) {
  int dev = 0, max_lds = 0;
  pwl_status st = device_ready(&dev, nullptr, &max_lds);
  if (st != PWL_OK) return st;
  const size_t need = std::max(pwl::finalize_lds_bytes(bp.N),
                               pwl::batch_table_lds_bytes(bp.N, pwl::map_cells_max(bp.N), true));
  if (need > (size_t)max_lds)
    return fail(PWL_ECAPACITY, "N = %d needs %zu bytes of LDS, the device offers %d", bp.N, need, max_lds);
  pwl::TableDev td;
  const int kcap = pwl::map_cells_max(bp.N);
  const size_t bytes = layout(&td, nullptr, bp.N, kcap, bp.G);
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, bytes);
  if (e != hipSuccess) return fail(PWL_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  layout(&td, static_cast<char*>(base), bp.N, kcap, bp.G);
  pwl_table* t = new pwl_table{dev, kcap, bp, td, base, bytes};
  e = hipEventCreateWithFlags(&t->built, hipEventDisableTiming);
  if (e == hipSuccess) e = pwl::launch_build(t->bp, t->td, static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipEventRecord(t->built, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    if (t->built) (void)hipEventDestroy(t->built);
    (void)hipFree(base);
    delete t;
    return fail(PWL_EHIP, "build launch failed: %s", hipGetErrorString(e));
  }
  *out = t;
  return PWL_OK;
}

}  // namespace

extern "C" {

pwl_status pwl_build(int32_t func, const double* params, int32_t nparams, double a, double b, int32_t N,
                     int32_t partition, int32_t values, void* stream, pwl_table** out) {
  if (out == nullptr) return fail(PWL_EINVAL, "out is NULL");
  *out = nullptr;
  pwl::BuildParams bp;
  pwl_status st = resolve_build(func, params, nparams, a, b, N, partition, values, &bp);
  if (st != PWL_OK) return st;
  return create_table(bp, stream, out);
}

}  // extern "C"

namespace {

// Fine cells for the prediction integrals: the density has |x - z|^(2/5)
// cusps at zeros of f'', so the trapezoid rule converges as dt^(7/5); 2^20
// cells give ~1e-8 relative accuracy, far below what moves N.
constexpr int kNormCells = 1 << 20;

}  // namespace

extern "C" {

pwl_status pwl_plan_tol(int32_t func, const double* params, int32_t nparams, double a, double b, double tol,
                        int32_t norm, int32_t values, void* stream, int32_t* N_out, int32_t* partition_out,
                        double* predicted_out) {
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(PWL_EINVAL, "tol must be finite and > 0");
  if (norm != PWL_NORM_L2 && norm != PWL_NORM_LINF) return fail(PWL_EINVAL, "unknown norm %d", norm);
  pwl::BuildParams bp;
  pwl_status st = resolve_build(func, params, nparams, a, b, 1, PWL_UNIFORM, values, &bp);
  if (st != PWL_OK) return st;
  int dev = 0;
  st = device_ready(&dev, nullptr);
  if (st != PWL_OK) return st;
  const int G = pwl::norm_blocks(kNormCells);
  void* scratch = nullptr;
  hipError_t e = hipMalloc(&scratch, sizeof(double) * (3 * (size_t)G + 3));
  if (e != hipSuccess) return fail(PWL_ENOMEM, "hipMalloc for the prediction integrals failed: %s", hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double h[3] = {0.0, 0.0, 0.0};
  e = pwl::launch_norms(bp.f, bp.a, bp.b, kNormCells, static_cast<double*>(scratch), s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h, static_cast<double*>(scratch) + 3 * G, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(PWL_EHIP, "prediction integrals failed: %s", hipGetErrorString(e));
  const double I25 = h[0], l2f2 = std::sqrt(h[1]), maxf2 = h[2], L = bp.b - bp.a;
  if (!std::isfinite(I25) || !std::isfinite(l2f2) || !std::isfinite(maxf2))
    return fail(PWL_EINVAL, "the second derivative is not finite on [a, b]");
  // predicted error = C / N^2 (Results 4-6, Sec. III-B2; L-infinity from the
  // interpolation remainder h^2 |f''| / 8 and the projection's h^2 |f''| / 12)
  const double r120 = std::sqrt(120.0), r6 = std::sqrt(6.0);
  double c_opt, c_uni;
  if (norm == PWL_NORM_L2) {
    c_opt = std::pow(I25, 2.5) / r120;
    c_uni = L * L * l2f2 / r120;
    if (values == PWL_PROJ) {
      c_opt /= r6;
      c_uni /= r6;
    }
  } else {
    const double k = (values == PWL_PROJ) ? 12.0 : 8.0;
    c_opt = std::pow(maxf2, 0.2) * I25 * I25 / k;
    c_uni = L * L * maxf2 / k;
  }
  auto need = [&](double c) -> double { return (c > 0.0) ? std::ceil(std::sqrt(c / tol)) : 1.0; };
  const double n_opt = std::max(1.0, need(c_opt)), n_uni = std::max(1.0, need(c_uni));
  // the optimal partition only when it needs fewer segments (its build costs more)
  const bool opt = n_opt < n_uni;
  const double n = opt ? n_opt : n_uni, c = opt ? c_opt : c_uni;
  if (n > PWL_MAX_N)
    return fail(PWL_ECAPACITY, "tol = %g needs N = %.0f segments (PWL_MAX_N = %d; the best at N = %d is %g)",
                tol, n, PWL_MAX_N, PWL_MAX_N, c / ((double)PWL_MAX_N * PWL_MAX_N));
  if (N_out) *N_out = (int32_t)n;
  if (partition_out) *partition_out = opt ? PWL_OPTIMAL : PWL_UNIFORM;
  if (predicted_out) *predicted_out = c / (n * n);
  return PWL_OK;
}

pwl_status pwl_build_tol(int32_t func, const double* params, int32_t nparams, double a, double b, double tol,
                         int32_t norm, int32_t values, void* stream, pwl_table** out) {
  if (out == nullptr) return fail(PWL_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t N = 0, partition = 0;
  pwl_status st = pwl_plan_tol(func, params, nparams, a, b, tol, norm, values, stream, &N, &partition, nullptr);
  if (st != PWL_OK) return st;
  return pwl_build(func, params, nparams, a, b, N, partition, values, stream, out);
}

pwl_status pwl_build_sampled(const double* f, const double* f2, int32_t S, double a, double b, int32_t N,
                             int32_t partition, int32_t values, void* stream, pwl_table** out) {
  if (out == nullptr) return fail(PWL_EINVAL, "out is NULL");
  *out = nullptr;
  if (f == nullptr || f2 == nullptr) return fail(PWL_EINVAL, "f and f2 must be non-NULL device arrays");
  if (S < 1) return fail(PWL_EINVAL, "S must be >= 1, got %d", S);
  // resolve with a stand-in function, then describe the samples
  pwl::BuildParams bp;
  pwl_status st = resolve_build(PWL_F_POLY, nullptr, 0, a, b, N, partition, values, &bp);
  if (st != PWL_OK) return st;
  bp.f.func = PWL_F_SAMPLED;
  bp.f.sf = f;
  bp.f.sf2 = f2;
  bp.f.S = S;
  bp.f.s_a = a;
  bp.f.s_h = (b - a) / (double)S;
  return create_table(bp, stream, out);
}

pwl_status pwl_rebuild(pwl_table* t, int32_t func, const double* params, int32_t nparams, double a,
                       double b, int32_t partition, int32_t values, void* stream) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (t->bp.f.func == PWL_F_SAMPLED)
    return fail(PWL_EINVAL, "a table built from samples cannot be rebuilt: build a new one");
  pwl::BuildParams bp;
  pwl_status st = resolve_build(func, params, nparams, a, b, t->bp.N, partition, values, &bp);
  if (st != PWL_OK) return st;
  if (bp.K > t->kcap)
    return fail(PWL_ECAPACITY, "rebuild needs %d map cells but the table holds %d", bp.K, t->kcap);
  st = check_table(t, nullptr);
  if (st != PWL_OK) return st;
  t->bp = bp;
  PWL_HIP(pwl::launch_build(t->bp, t->td, static_cast<hipStream_t>(stream)));
  PWL_HIP(hipEventRecord(t->built, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_table_check(const pwl_table* t, void* stream, int32_t* flags) {
  pwl_status st = check_table(t, nullptr);
  if (st != PWL_OK) return st;
  uint32_t host = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PWL_HIP(hipMemcpyAsync(&host, t->td.status, sizeof(host), hipMemcpyDeviceToHost, s));
  PWL_HIP(hipStreamSynchronize(s));
  if (flags) *flags = (int32_t)host;
  if (host & PWL_FLAG_KNOTS_COLLAPSED)
    return fail(PWL_EKNOTS, "FP32 knots are not strictly increasing (N too large for the domain)");
  return PWL_OK;
}

pwl_status pwl_table_info(const pwl_table* t, int32_t* N, double* a, double* b, int32_t* partition,
                          int32_t* values, int32_t* map_cells, int32_t* flags) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (flags) {
    // the flags of the table's last build: the library's own stream waits
    // for that build only (an event recorded after it), then reads the word
    pwl_status st = check_table(t, nullptr);
    if (st != PWL_OK) return st;
    uint32_t host = 0;
    hipStream_t aux = g_aux[t->device];
    PWL_HIP(hipStreamWaitEvent(aux, t->built, 0));
    PWL_HIP(hipMemcpyAsync(&host, t->td.status, sizeof(host), hipMemcpyDeviceToHost, aux));
    PWL_HIP(hipStreamSynchronize(aux));
    *flags = (int32_t)host;
  }
  if (N) *N = t->bp.N;
  if (a) *a = t->bp.a;
  if (b) *b = t->bp.b;
  if (partition) *partition = t->bp.partition;
  if (values) *values = t->bp.values;
  if (map_cells) *map_cells = t->bp.K;
  return PWL_OK;
}

pwl_status pwl_table_download(const pwl_table* t, float* knots, float* values, double* knots64,
                              double* values64, void* stream) {
  pwl_status st = check_table(t, nullptr);
  if (st != PWL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n1 = (size_t)t->bp.N + 1;
  if (knots) PWL_HIP(hipMemcpyAsync(knots, t->td.knots, n1 * sizeof(float), hipMemcpyDeviceToHost, s));
  if (values) PWL_HIP(hipMemcpyAsync(values, t->td.values, n1 * sizeof(float), hipMemcpyDeviceToHost, s));
  if (knots64)
    PWL_HIP(hipMemcpyAsync(knots64, t->td.knots64, n1 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (values64)
    PWL_HIP(hipMemcpyAsync(values64, t->td.values64, n1 * sizeof(double), hipMemcpyDeviceToHost, s));
  PWL_HIP(hipStreamSynchronize(s));
  return PWL_OK;
}

void pwl_table_free(pwl_table* t) {
  if (t == nullptr) return;
  if (t->part != nullptr) {
    // stream-ordered memory: released after its last user, then waited for
    (void)hipEventSynchronize(t->part_used);
    (void)hipFreeAsync(t->part, g_aux[t->device]);
    (void)hipStreamSynchronize(g_aux[t->device]);
  }
  if (t->part_used) (void)hipEventDestroy(t->part_used);
  if (t->built) (void)hipEventDestroy(t->built);
  (void)hipFree(t->base);
  delete t;
}

pwl_status pwl_eval(const pwl_table* t, const float* v_override, const float* x, float* y, int64_t n,
                    void* stream) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (n == 0) return PWL_OK;
  if (x == nullptr || y == nullptr) return fail(PWL_EINVAL, "x and y must be non-NULL");
  int num_cu = 1;
  pwl_status st = check_table(t, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_eval(eval_view(t), v_override, x, y, n, num_cu, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_eval_backward(const pwl_table* t, const float* v_override, const float* x, const float* g,
                             float* y, float* dx, float* dv, int64_t n, void* stream) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (y == nullptr && dx == nullptr && dv == nullptr)
    return fail(PWL_EINVAL, "at least one of y, dx, dv must be non-NULL");
  if (n > 0 && (x == nullptr || g == nullptr)) return fail(PWL_EINVAL, "x and g must be non-NULL");
  int num_cu = 1;
  if (n == 0 && dv == nullptr) return PWL_OK;
  pwl_status st = check_table(t, &num_cu);
  if (st != PWL_OK) return st;
  const pwl::EvalTable e = eval_view(t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dv == nullptr || n == 0) {
    PWL_HIP(pwl::launch_eval_backward(e, v_override, x, g, y, dx, dv, nullptr, n, num_cu, s));
    return PWL_OK;
  }
  // The partial-sum rows: grown in stream order on the caller's stream (the
  // old rows are released once their last user - on whatever stream - has
  // finished), never by a device-wide synchronisation.
  std::lock_guard<std::mutex> lock(t->part_mu);
  const size_t need = pwl::backward_workspace_floats(e, x, g, y, dx, n, num_cu);
  if (need > t->part_cap) {
    if (t->part != nullptr) {
      PWL_HIP(hipStreamWaitEvent(s, t->part_used, 0));
      PWL_HIP(hipFreeAsync(t->part, s));
      t->part = nullptr;
      t->part_cap = 0;
    }
    if (t->part_used == nullptr) PWL_HIP(hipEventCreateWithFlags(&t->part_used, hipEventDisableTiming));
    void* p = nullptr;
    hipError_t me = hipMallocAsync(&p, need * sizeof(float), s);
    if (me != hipSuccess)
      return fail(PWL_ENOMEM, "hipMallocAsync(%zu) for the dL/dv partial sums failed: %s", need * sizeof(float),
                  hipGetErrorString(me));
    t->part = static_cast<float*>(p);
    t->part_cap = need;
  }
  PWL_HIP(pwl::launch_eval_backward(e, v_override, x, g, y, dx, dv, t->part, n, num_cu, s));
  PWL_HIP(hipEventRecord(t->part_used, s));
  return PWL_OK;
}

pwl_status pwl_eval_backward_noalloc(const pwl_table* t, const float* v_override, const float* x, const float* g,
                                     float* y, float* dx, float* dv, int64_t n, void* stream) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (y == nullptr && dx == nullptr && dv == nullptr)
    return fail(PWL_EINVAL, "at least one of y, dx, dv must be non-NULL");
  if (n > 0 && (x == nullptr || g == nullptr)) return fail(PWL_EINVAL, "x and g must be non-NULL");
  if (n == 0 && dv == nullptr) return PWL_OK;
  int num_cu = 1, dev = 0;
  pwl_status st = check_table(t, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(hipGetDevice(&dev));
  const pwl::EvalTable e = eval_view(t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* part = nullptr;
  if (dv != nullptr && n > 0) {
    // the same launch shape (and so the same rows) as pwl_eval_backward
    const size_t need = pwl::backward_workspace_floats(e, x, g, y, dx, n, num_cu);
    if (need > kScratchFloats)
      return fail(PWL_ECAPACITY,
                  "pwl_eval_backward_noalloc: the dL/dv partial sums need %zu floats (workgroups x (N + 1)), "
                  "above the %zu of its fixed device scratch; use pwl_eval_backward or a smaller backward "
                  "launch shape",
                  need, kScratchFloats);
    part = g_scratch[dev];
  }
  PWL_HIP(pwl::launch_eval_backward(e, v_override, x, g, y, dx, dv, part, n, num_cu, s));
  return PWL_OK;
}

pwl_status pwl_locate(const pwl_table* t, const float* x, int32_t* seg, int64_t n, void* stream) {
  if (t == nullptr) return fail(PWL_EINVAL, "table is NULL");
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (n == 0) return PWL_OK;
  if (x == nullptr || seg == nullptr) return fail(PWL_EINVAL, "x and seg must be non-NULL");
  int num_cu = 1;
  pwl_status st = check_table(t, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_locate(eval_view(t), x, seg, n, num_cu, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_direct_gaussian(const float* x, float* y, int64_t n, float s, float amp, int32_t fast,
                               void* stream) {
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (!(s > 0.0f) || !std::isfinite(s) || !std::isfinite(amp))
    return fail(PWL_EINVAL, "s must be finite and > 0, amp finite");
  if (n == 0) return PWL_OK;
  if (x == nullptr || y == nullptr) return fail(PWL_EINVAL, "x and y must be non-NULL");
  int num_cu = 1;
  pwl_status st = device_ready(nullptr, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_direct_gaussian(x, y, n, s, amp, fast, num_cu, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_direct_eval(int32_t func, const double* params, int32_t nparams, const float* x, float* y, int64_t n,
                           void* stream) {
  pwl::FuncDesc f;
  pwl_status st = resolve_func(func, params, nparams, &f);
  if (st != PWL_OK) return st;
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (n == 0) return PWL_OK;
  if (x == nullptr || y == nullptr) return fail(PWL_EINVAL, "x and y must be non-NULL");
  int num_cu = 1;
  st = device_ready(nullptr, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_direct_func(f, x, y, n, num_cu, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_copy(const float* src, float* dst, int64_t n, void* stream) {
  if (n < 0) return fail(PWL_EINVAL, "n must be >= 0");
  if (n == 0) return PWL_OK;
  if (src == nullptr || dst == nullptr) return fail(PWL_EINVAL, "src and dst must be non-NULL");
  int num_cu = 1;
  pwl_status st = device_ready(nullptr, &num_cu);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_copy(src, dst, n, num_cu, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_kde(const pwl_table* t, int32_t mode, const void* frame, const void* hist, int32_t H, int32_t W,
                   int32_t T, int32_t r, const float* sigma, float* out, void* stream) {
  if (mode != PWL_KDE_TABLE && mode != PWL_KDE_EXPF && mode != PWL_KDE_FAST_EXPF)
    return fail(PWL_EINVAL, "unknown kde mode %d", mode);
  if (H < 1 || W < 1 || T < 1) return fail(PWL_EINVAL, "need H, W, T >= 1 (got %d, %d, %d)", H, W, T);
  if (r < 0 || r > 32) return fail(PWL_EINVAL, "window radius must be in [0, 32], got %d", r);
  if (frame == nullptr || hist == nullptr || out == nullptr || sigma == nullptr)
    return fail(PWL_EINVAL, "frame, hist, sigma and out must be non-NULL");
  for (int c = 0; c < 3; ++c)
    if (!(sigma[c] > 0.0f) || !std::isfinite(sigma[c])) return fail(PWL_EINVAL, "sigma[%d] must be > 0", c);
  if (mode == PWL_KDE_TABLE && t == nullptr) return fail(PWL_EINVAL, "the table mode needs a table");
  int num_cu = 1;
  pwl_status st = (mode == PWL_KDE_TABLE) ? check_table(t, &num_cu) : device_ready(nullptr, &num_cu);
  if (st != PWL_OK) return st;
  pwl::EvalTable e{};
  if (mode == PWL_KDE_TABLE) e = eval_view(t);
  PWL_HIP(pwl::launch_kde(e, mode, frame, hist, H, W, T, r, sigma, out, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

// ---- batches ---------------------------------------------------------------

}  // extern "C"

namespace {

// Vector iterations per slice, forward and backward.  Longer slices stage
// less often but stream worse: on the 4096-table workload the forward
// measured fastest at 2 (3: +1%, 4: +6%), the fused backward at 4 (2: +10%,
// 8: +2%), and slices lengthened in proportion to their table's LDS bytes
// (to stage big tables less often) slower still.
constexpr int kSliceIterations[2] = {2, 4};

struct ClassPlan {
  std::vector<pwl::BatchRun> runs;
  std::vector<pwl::BatchGroup> groups;
  size_t lds = 16;
};

// The points in slices of `slice` points from point 0 on (the last one
// shorter), each slice the runs of the tables it meets.  A slice whose
// tables need more than `cap` bytes of LDS together - their images, a
// contiguous span of the arena, and (backward) one FP64 dL/dv region per
// table after them - becomes several groups, split at a table.  The kernels
// deal the groups to their workgroups round-robin, in the order below.
ClassPlan plan_slices(const int64_t* offsets, int T, const std::vector<int64_t>& img_word,
                      const std::vector<int32_t>& nvec, const std::vector<int32_t>& Ns, bool backward,
                      int64_t slice, size_t cap) {
  ClassPlan p;
  const int64_t total = offsets[T];
  auto dvw = [&](int u) { return backward ? (int64_t)pwl::batch_dv_words(Ns[u]) : 0; };
  auto close = [&](int q, int64_t img0, int64_t dv_words) {
    const int q1 = (int)p.runs.size();
    if (q1 == q) return;
    const int last = p.runs[q1 - 1].table;
    pwl::BatchGroup g{};
    g.img = img0;
    g.nwords = (int32_t)(img_word[last] + nvec[last] - img0);
    g.r0 = q;
    g.r1 = q1;
    g.dv_lds = g.nwords;
    g.dv_words = (int32_t)dv_words;
    int64_t cum = 0;
    for (int k = q; k < q1; ++k) {
      pwl::BatchRun& r = p.runs[k];
      r.img_lds = (int32_t)(img_word[r.table] - img0);
      r.dv_lds = backward ? (int32_t)(g.nwords + cum) : 0;
      cum += dvw(r.table);
    }
    p.lds = std::max(p.lds, (size_t)(16 * ((size_t)g.nwords + (size_t)dv_words)));
    p.groups.push_back(g);
  };
  int t0 = 0;
  for (int64_t s0 = 0; s0 < total; s0 += slice) {
    const int64_t s1 = std::min(total, s0 + slice);
    while (offsets[t0 + 1] <= s0) ++t0;   // the table holding point s0
    int q = (int)p.runs.size();
    int64_t img0 = -1, dv_words = 0;
    for (int u = t0; u < T && offsets[u] < s1; ++u) {
      if (offsets[u + 1] == offsets[u]) continue;   // no points
      if (img0 >= 0 && (size_t)(16 * (img_word[u] + nvec[u] - img0 + dv_words + dvw(u))) > cap) {
        close(q, img0, dv_words);
        q = (int)p.runs.size();
        img0 = -1;
        dv_words = 0;
      }
      if (img0 < 0) img0 = img_word[u];
      dv_words += dvw(u);
      pwl::BatchRun r{};
      r.table = u;
      r.begin = std::max(s0, offsets[u]);
      r.end = std::min(s1, offsets[u + 1]);
      p.runs.push_back(r);
    }
    close(q, img0, dv_words);
  }
  // Deal each run of 8 consecutive units to one XCD: launch position
  // 64 c + 8 j + i takes unit 64 c + 8 i + j (workgroups go to the XCDs
  // round-robin, so position p runs on XCD p mod 8), keeping every block of
  // 64 positions a window of 64 consecutive units.  A table's consecutive
  // slices then read its image through one L2: the 4096-table forward
  // measured 382.5 -> 375.8 us, the fused backward unchanged.
  const int G = (int)p.groups.size(), full = G / 64 * 64;
  std::vector<pwl::BatchGroup> order(p.groups);
  for (int pos = 0; pos < full; ++pos) {
    const int c = pos / 64, j = (pos / 8) % 8, i = pos % 8;
    order[pos] = p.groups[64 * c + 8 * i + j];
  }
  p.groups.swap(order);
  return p;
}

}  // namespace

extern "C" {

pwl_status pwl_batch_create(const pwl_table* const* tables, int32_t T, const int64_t* offsets, void* stream,
                            pwl_batch** out) {
  if (out == nullptr) return fail(PWL_EINVAL, "out is NULL");
  *out = nullptr;
  if (tables == nullptr || offsets == nullptr) return fail(PWL_EINVAL, "tables and offsets must be non-NULL");
  if (T < 1) return fail(PWL_EINVAL, "T must be >= 1");
  if (offsets[0] != 0) return fail(PWL_EINVAL, "offsets[0] must be 0");
  for (int i = 0; i < T; ++i) {
    if (tables[i] == nullptr) return fail(PWL_EINVAL, "tables[%d] is NULL", i);
    if (offsets[i + 1] < offsets[i]) return fail(PWL_EINVAL, "offsets must be non-decreasing (at %d)", i);
  }
  int dev = 0, num_cu = 1;
  pwl_status st = device_ready(&dev, &num_cu);
  if (st != PWL_OK) return st;
  for (int i = 0; i < T; ++i)
    if (tables[i]->device != dev)
      return fail(PWL_EINVAL, "tables[%d] lives on device %d, current is %d", i, tables[i]->device, dev);
  // the images in table order, each on a 256-byte boundary of the arena
  std::vector<int32_t> nvec(T), Ns(T);
  std::vector<int64_t> img_word(T);
  int64_t arena_words = 0;
  for (int i = 0; i < T; ++i) {
    Ns[i] = tables[i]->bp.N;
    nvec[i] = pwl::image_words(tables[i]->bp.N, tables[i]->bp.K);
    img_word[i] = arena_words;
    arena_words += (nvec[i] + 15) / 16 * 16;
  }
  int max_lds = 0;
  (void)device_ready(nullptr, nullptr, &max_lds);
  const size_t cap = std::min<size_t>((size_t)max_lds, 160 * 1024);
  // slices of whole vector iterations of each kernel's current shape; a
  // persistent grid of wg_per_cu workgroups per CU (no more than slices)
  const pwl::LaunchConfig cfg[2] = {pwl::get_launch(PWL_KERNEL_BATCH), pwl::get_launch(PWL_KERNEL_BATCH_BACKWARD)};
  ClassPlan plans[2];
  int grids[2];
  for (int dir = 0; dir < 2; ++dir) {
    const int64_t slice = (int64_t)kSliceIterations[dir] * 4 * cfg[dir].block * cfg[dir].unroll;
    plans[dir] = plan_slices(offsets, T, img_word, nvec, Ns, dir == 1, slice, cap);
    const int64_t ng = (int64_t)plans[dir].groups.size();
    grids[dir] = (int)std::max<int64_t>(1, std::min<int64_t>(ng, (int64_t)num_cu * std::max(1, cfg[dir].wg_per_cu)));
  }
  // the backward's partial dL/dv sums: N + 1 per run; per table its runs'
  // offsets in slice order, and its range of the concatenated gradient
  std::vector<int64_t> tab_dv(T + 1, 0);
  for (int i = 0; i < T; ++i) tab_dv[i + 1] = tab_dv[i] + Ns[i] + 1;
  std::vector<int32_t> tab_first(T + 1, 0);
  int64_t part_len = 0;
  for (pwl::BatchRun& r : plans[1].runs) {
    r.part = part_len;
    part_len += Ns[r.table] + 1;
    ++tab_first[r.table + 1];
  }
  for (int i = 0; i < T; ++i) tab_first[i + 1] += tab_first[i];
  std::vector<int64_t> tab_part(std::max<size_t>(1, plans[1].runs.size()));
  {
    std::vector<int32_t> fill(tab_first.begin(), tab_first.end() - 1);
    for (const pwl::BatchRun& r : plans[1].runs) tab_part[fill[r.table]++] = r.part;
  }
  // one allocation: tables, their deepest map cells, the image arena, the
  // runs and work units of the forward and the backward launch, then the
  // backward's partial sums and their per-table lists
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  const size_t o_tab = take(sizeof(pwl::BatchTable) * T);
  const size_t o_maxc = take(sizeof(int32_t) * T);
  const size_t o_arena = take(16 * (size_t)std::max<int64_t>(1, arena_words));
  size_t o_runs[2], o_grp[2];
  for (int dir = 0; dir < 2; ++dir) {
    o_runs[dir] = take(sizeof(pwl::BatchRun) * std::max<size_t>(1, plans[dir].runs.size()));
    o_grp[dir] = take(sizeof(pwl::BatchGroup) * std::max<size_t>(1, plans[dir].groups.size()));
  }
  const size_t o_part = take(sizeof(float) * (size_t)std::max<int64_t>(1, part_len));
  const size_t o_tpart = take(sizeof(int64_t) * tab_part.size());
  const size_t o_tfirst = take(sizeof(int32_t) * (T + 1));
  const size_t o_tdv = take(sizeof(int64_t) * (T + 1));
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, off);
  if (e != hipSuccess) return fail(PWL_ENOMEM, "hipMalloc(%zu) failed: %s", off, hipGetErrorString(e));
  char* b = static_cast<char*>(base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<pwl::BatchTable> hb(T);
  for (int i = 0; i < T; ++i) {
    hb[i].t = eval_view(tables[i]);
    hb[i].img = reinterpret_cast<float4*>(b + o_arena) + img_word[i];
    hb[i].nvec = nvec[i];
    hb[i].pad = 0;
  }
  // images and deepest cells on the device, the cells back to the host
  std::vector<int32_t> maxc(T, 0);
  int32_t* d_maxc = reinterpret_cast<int32_t*>(b + o_maxc);
  e = hipMemcpyAsync(b + o_tab, hb.data(), sizeof(pwl::BatchTable) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = pwl::launch_batch_pack(reinterpret_cast<pwl::BatchTable*>(b + o_tab), T, d_maxc, s);
  if (e == hipSuccess) e = hipMemcpyAsync(maxc.data(), d_maxc, sizeof(int32_t) * T, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  // complete the run descriptors and upload the plans
  pwl_batch* bt = new pwl_batch{};
  for (int dir = 0; dir < 2; ++dir) {
    {
      ClassPlan& p = plans[dir];
      for (pwl::BatchRun& r : p.runs) {
        const pwl_table* t = tables[r.table];
        r.nvec = nvec[r.table];
        r.N = t->bp.N;
        r.K = t->bp.K;
        r.a32 = t->bp.a32;
        r.b32 = t->bp.b32;
        r.scale32 = t->bp.scale32;
        r.maxc = maxc[r.table];
      }
      for (pwl::BatchGroup& g : p.groups) {
        g.maxc = 0;
        for (int k = g.r0; k < g.r1; ++k) g.maxc = std::max(g.maxc, p.runs[k].maxc);
      }
      if (e == hipSuccess && !p.runs.empty())
        e = hipMemcpyAsync(b + o_runs[dir], p.runs.data(), sizeof(pwl::BatchRun) * p.runs.size(),
                           hipMemcpyHostToDevice, s);
      if (e == hipSuccess && !p.groups.empty())
        e = hipMemcpyAsync(b + o_grp[dir], p.groups.data(), sizeof(pwl::BatchGroup) * p.groups.size(),
                           hipMemcpyHostToDevice, s);
      pwl::BatchPlan& d = dir ? bt->bl.bwd : bt->bl.fwd;
      const int32_t ngroups = (int32_t)p.groups.size();
      d = pwl::BatchPlan{reinterpret_cast<pwl::BatchRun*>(b + o_runs[dir]),
                         reinterpret_cast<pwl::BatchGroup*>(b + o_grp[dir]),
                         reinterpret_cast<const float4*>(b + o_arena), grids[dir], ngroups,
                         (int32_t)p.runs.size(), p.lds};
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + o_tpart, tab_part.data(), sizeof(int64_t) * tab_part.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + o_tfirst, tab_first.data(), sizeof(int32_t) * (T + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + o_tdv, tab_dv.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(base);
    delete bt;
    return fail(PWL_EHIP, "batch upload failed: %s", hipGetErrorString(e));
  }
  bt->device = dev;
  bt->T = T;
  bt->npoints = offsets[T];
  bt->base = base;
  bt->bl.dv_len = tab_dv[T];
  bt->bl.T = T;
  bt->bl.max_n = *std::max_element(Ns.begin(), Ns.end());
  bt->bl.part = reinterpret_cast<float*>(b + o_part);
  bt->bl.tab_part = reinterpret_cast<const int64_t*>(b + o_tpart);
  bt->bl.tab_first = reinterpret_cast<const int32_t*>(b + o_tfirst);
  bt->bl.tab_dv = reinterpret_cast<const int64_t*>(b + o_tdv);
  *out = bt;
  return PWL_OK;
}

}  // extern "C"

namespace {

pwl_status check_batch(const pwl_batch* bt) {
  if (bt == nullptr) return fail(PWL_EINVAL, "batch is NULL");
  int dev = 0;
  pwl_status st = device_ready(&dev, nullptr);
  if (st != PWL_OK) return st;
  if (dev != bt->device)
    return fail(PWL_EINVAL, "batch lives on device %d but device %d is current", bt->device, dev);
  return PWL_OK;
}

pwl_status check_batch_args(const pwl_batch* bt, const float* x, const float* g, float* y, float* dx, float* dv) {
  if (bt->npoints > 0 && x == nullptr) return fail(PWL_EINVAL, "x must be non-NULL");
  if (g == nullptr) {
    if (bt->npoints > 0 && y == nullptr) return fail(PWL_EINVAL, "y must be non-NULL");
  } else {
    if (dv == nullptr) return fail(PWL_EINVAL, "the batched backward needs dv");
  }
  (void)dx;
  return PWL_OK;
}

}  // namespace

extern "C" {

pwl_status pwl_batch_eval(pwl_batch* bt, const float* x, float* y, void* stream) {
  pwl_status st = check_batch(bt);
  if (st != PWL_OK) return st;
  st = check_batch_args(bt, x, nullptr, y, nullptr, nullptr);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_batch(bt->bl, x, nullptr, y, nullptr, nullptr, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_batch_eval_backward(pwl_batch* bt, const float* x, const float* g, float* y, float* dx, float* dv,
                                   void* stream) {
  pwl_status st = check_batch(bt);
  if (st != PWL_OK) return st;
  if (g == nullptr && bt->npoints > 0) return fail(PWL_EINVAL, "g must be non-NULL");
  if (dv == nullptr) return fail(PWL_EINVAL, "the batched backward needs dv");
  // With no points g is never read; any non-NULL stand-in selects the backward.
  const float* gg = (g != nullptr) ? g : dv;
  st = check_batch_args(bt, x, gg, y, dx, dv);
  if (st != PWL_OK) return st;
  PWL_HIP(pwl::launch_batch(bt->bl, x, gg, y, dx, dv, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_batch_capture(pwl_batch* bt, const float* x, const float* g, float* y, float* dx, float* dv,
                             void* stream) {
  pwl_status st = check_batch(bt);
  if (st != PWL_OK) return st;
  st = check_batch_args(bt, x, g, y, dx, dv);
  if (st != PWL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PWL_HIP(hipStreamSynchronize(s));
  hipStream_t cs = nullptr;
  PWL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = pwl::launch_batch(bt->bl, x, g, y, dx, dv, cs);
    e = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = le;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(PWL_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->graph = graph;
  bt->exec = exec;
  return PWL_OK;
}

pwl_status pwl_batch_replay(pwl_batch* bt, void* stream) {
  pwl_status st = check_batch(bt);
  if (st != PWL_OK) return st;
  if (bt->exec == nullptr) return fail(PWL_EINVAL, "no captured graph: call pwl_batch_capture first");
  PWL_HIP(hipGraphLaunch(bt->exec, static_cast<hipStream_t>(stream)));
  return PWL_OK;
}

pwl_status pwl_batch_info(const pwl_batch* bt, int32_t* T, int64_t* npoints, int64_t* dv_len, int32_t* grid_fwd,
                          int32_t* grid_bwd, int32_t* runs_fwd, int32_t* runs_bwd) {
  if (bt == nullptr) return fail(PWL_EINVAL, "batch is NULL");
  if (T) *T = bt->T;
  if (npoints) *npoints = bt->npoints;
  if (dv_len) *dv_len = bt->bl.dv_len;
  if (grid_fwd) *grid_fwd = bt->bl.fwd.grid;
  if (grid_bwd) *grid_bwd = bt->bl.bwd.grid;
  if (runs_fwd) *runs_fwd = bt->bl.fwd.nruns;
  if (runs_bwd) *runs_bwd = bt->bl.bwd.nruns;
  return PWL_OK;
}

void pwl_batch_free(pwl_batch* bt) {
  if (bt == nullptr) return;
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  (void)hipFree(bt->base);
  delete bt;
}

pwl_status pwl_set_launch(int32_t kernel, int32_t unroll, int32_t block, int32_t wg_per_cu) {
  if (pwl::set_launch(kernel, unroll, block, wg_per_cu) != hipSuccess)
    return fail(PWL_EINVAL, "invalid launch shape (kernel %d, unroll %d, block %d, wg_per_cu %d)", kernel,
                unroll, block, wg_per_cu);
  return PWL_OK;
}

pwl_status pwl_set_locate(int32_t mode) {
  if (pwl::set_locate(mode) != hipSuccess) return fail(PWL_EINVAL, "unknown locate mode %d", mode);
  return PWL_OK;
}

int32_t pwl_get_locate(void) { return pwl::get_locate(); }

pwl_status pwl_set_records(int32_t layout) {
  if (pwl::set_records(layout) != hipSuccess) return fail(PWL_EINVAL, "unknown record layout %d", layout);
  return PWL_OK;
}

int32_t pwl_get_records(void) { return pwl::get_records(); }

pwl_status pwl_get_launch(int32_t kernel, int32_t* unroll, int32_t* block, int32_t* wg_per_cu) {
  if (kernel < 0 || kernel > 3) return fail(PWL_EINVAL, "unknown kernel family %d", kernel);
  const pwl::LaunchConfig c = pwl::get_launch(kernel);
  if (unroll) *unroll = c.unroll;
  if (block) *block = c.block;
  if (wg_per_cu) *wg_per_cu = c.wg_per_cu;
  return PWL_OK;
}

}  // extern "C"
