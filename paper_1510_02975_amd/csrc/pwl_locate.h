// Segment locate (step 1 of Algorithm 1, Sec. IV) through a uniform index map.
//
// The paper locates x in a non-uniform partition with an O(log N) binary
// search (Sec. IV) unrolled into selects (Sec. V).  Here the domain is cut
// into K equal cells; cell(x) is monotone non-decreasing in x because each
// FP32 operation below is monotone, so for every knot x_k with
// cell(x_k) < cell(x) we have x_k <= x, and for every knot with
// cell(x_k) > cell(x) we have x_k > x.  Storing, per cell u,
//   lo[u]    = #{interior knots k : cell(x_k) <  u}
//   count[u] = #{interior knots k : cell(x_k) == u}
// the segment of x is lo[u] plus the number of the count[u] knots of its
// cell that are <= x: exact, with no rounding slack, as long as the map is
// built with this very function.
#pragma once

#include <hip/hip_runtime.h>

namespace pwl {

__device__ __forceinline__ int map_cell(float x, float a32, float scale32, int K) {
#pragma clang fp contract(off)
  float t = (x - a32) * scale32;
  // fmaxf returns the non-NaN operand, so NaN x lands in cell 0.
  t = fminf(fmaxf(t, 0.0f), (float)(K - 1));
  return (int)t;
}

// Segment index in [0, N-1] of x (clamped to the domain).  knots[k] holds the
// interior knot x_k for 1 <= k <= N-1 and +inf for k >= N; cells[u] holds
// lo | count << 16.
template <typename KnotPtr, typename CellPtr>
__device__ __forceinline__ int locate_segment(float x, KnotPtr knots, CellPtr cells, float a32,
                                              float scale32, int K) {
  const int u = map_cell(x, a32, scale32, K);
  const uint32_t e = cells[u];
  int seg = (int)(e & 0xffffu);
  const int cnt = (int)(e >> 16);
  const int lo = seg;
  for (int j = 1; j <= cnt; ++j) seg += (x >= knots[lo + j]) ? 1 : 0;
  return seg;
}

}  // namespace pwl
