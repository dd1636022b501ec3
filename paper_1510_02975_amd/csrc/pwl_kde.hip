// Sample application of the approximation (Sec. VI-A): per-pixel sums of
// Gaussian kernels of a nonparametric background model.  For pixel (y, x)
// of the current frame and every pixel (y', x') of the (2r+1) x (2r+1)
// window (clamped to the image) in each of T reference frames,
//   L(y, x) = 1 / (T (2r+1)^2) * sum prod_{c = R, G, B} g((f_c - h_c) / sigma_c),
// with g(u) = exp(-u^2 / 2) evaluated either through a CPWL table (staged in
// LDS; |u| when the table's domain starts at 0) or with expf / __expf - the
// comparison the paper makes for this application.  One thread per pixel,
// 16 x 16 pixel tiles; the reference pixels of a tile's windows are shared
// by neighbouring threads and come from L1/L2.  The sum is accumulated in
// FP64 so that only the kernel evaluations round.
#include <hip/hip_runtime.h>

#include "pwl_internal.h"
#include "pwl_stream.h"

namespace pwl {

namespace {

using namespace stream;

constexpr int kTile = 16;

template <int MODE, int MAXC>
__device__ __forceinline__ float kernel_g(float u, const EvalTable& t, const Smem& s) {
  if (MODE == PWL_KDE_TABLE) return eval_point<MAXC>(t.a32 >= 0.0f ? fabsf(u) : u, t, s);
  if (MODE == PWL_KDE_EXPF) return expf(-0.5f * u * u);
  return __expf(-0.5f * u * u);
}

template <int MODE, int MAXC>
__device__ __forceinline__ void kde_pixel(const EvalTable& t, const Smem& s, const uchar4* __restrict__ frame,
                                          const uchar4* __restrict__ hist, int H, int W, int T, int r,
                                          float is0, float is1, float is2, float* __restrict__ out, int y,
                                          int x) {
  const uchar4 p = frame[(int64_t)y * W + x];
  const float f0 = (float)p.x, f1 = (float)p.y, f2 = (float)p.z;
  double sum = 0.0;
  for (int k = 0; k < T; ++k) {
    const uchar4* __restrict__ hk = hist + (int64_t)k * H * W;
    for (int dy = -r; dy <= r; ++dy) {
      const int yy = min(max(y + dy, 0), H - 1);
      for (int dx = -r; dx <= r; ++dx) {
        const int xx = min(max(x + dx, 0), W - 1);
        const uchar4 h = hk[(int64_t)yy * W + xx];
        const float g = kernel_g<MODE, MAXC>((f0 - (float)h.x) * is0, t, s) *
                        kernel_g<MODE, MAXC>((f1 - (float)h.y) * is1, t, s) *
                        kernel_g<MODE, MAXC>((f2 - (float)h.z) * is2, t, s);
        sum += (double)g;
      }
    }
  }
  const int w = 2 * r + 1;
  out[(int64_t)y * W + x] = (float)(sum / ((double)T * w * w));
}

template <int MODE>
__global__ __launch_bounds__(kTile * kTile) void k_kde(EvalTable t, const uchar4* __restrict__ frame,
                                                       const uchar4* __restrict__ hist, int H, int W, int T,
                                                       int r, float is0, float is1, float is2,
                                                       float* __restrict__ out) {
  extern __shared__ float4 lds_f4[];
  Smem s{};
  if (MODE == PWL_KDE_TABLE) {
    s = carve(lds_f4, t.N, t.K, false);
    stage_table(t, nullptr, s);
    __syncthreads();
  }
  const int x = blockIdx.x * kTile + (int)(threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (int)(threadIdx.x / kTile);
  if (x >= W || y >= H) return;
  if (MODE != PWL_KDE_TABLE) {
    kde_pixel<MODE, 1>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x);
    return;
  }
  switch (t.meta[1]) {
    case 0:
    case 1: kde_pixel<MODE, 1>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x); break;
    case 2: kde_pixel<MODE, 2>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x); break;
    case 3: kde_pixel<MODE, 3>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x); break;
    case 4: kde_pixel<MODE, 4>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x); break;
    default: kde_pixel<MODE, 0>(t, s, frame, hist, H, W, T, r, is0, is1, is2, out, y, x); break;
  }
}

}  // namespace

hipError_t launch_kde(const EvalTable& t, int mode, const void* frame, const void* hist, int H, int W, int T,
                      int r, const float* sigma, float* out, hipStream_t s) {
  const dim3 grid((W + kTile - 1) / kTile, (H + kTile - 1) / kTile), block(kTile * kTile);
  const float is0 = 1.0f / sigma[0], is1 = 1.0f / sigma[1], is2 = 1.0f / sigma[2];
  const uchar4* f = static_cast<const uchar4*>(frame);
  const uchar4* h = static_cast<const uchar4*>(hist);
  switch (mode) {
    case PWL_KDE_TABLE:
      hipLaunchKernelGGL(k_kde<PWL_KDE_TABLE>, grid, block, eval_lds_bytes(t.N, t.K, false), s, t, f, h, H, W, T,
                         r, is0, is1, is2, out);
      break;
    case PWL_KDE_EXPF:
      hipLaunchKernelGGL(k_kde<PWL_KDE_EXPF>, grid, block, 0, s, t, f, h, H, W, T, r, is0, is1, is2, out);
      break;
    default:
      hipLaunchKernelGGL(k_kde<PWL_KDE_FAST_EXPF>, grid, block, 0, s, t, f, h, H, W, T, r, is0, is1, is2, out);
      break;
  }
  return hipGetLastError();
}

hipError_t configure_kde_kernels(int max_lds) {
  const int lim = max_lds < 160 * 1024 ? max_lds : 160 * 1024;
  return hipFuncSetAttribute((const void*)k_kde<PWL_KDE_TABLE>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

}  // namespace pwl
