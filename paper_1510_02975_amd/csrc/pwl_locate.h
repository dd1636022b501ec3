// Segment locate (the first part of Algorithm 1, Sec. IV) through a uniform index map.
//
// The paper locates x in a non-uniform partition with an O(log N) binary
// search (Sec. IV) unrolled into selects (Sec. V).  Here the domain is cut
// into K equal cells; cell(x) is monotone non-decreasing in x because each
// FP32 operation below is monotone, so for every knot x_k with
// cell(x_k) < cell(x) we have x_k <= x, and for every knot with
// cell(x_k) > cell(x) we have x_k > x.  Storing, per cell u,
//   lo[u] = #{interior knots k : cell(x_k) < u}     (lo[K] = N - 1),
// cell u holds the count[u] = lo[u+1] - lo[u] knots x_{lo[u]+1} ..., and the
// segment of x is lo[u] plus the number of those knots that are <= x:
// exact, with no rounding slack, as long as the map is built with this very
// function.
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

}  // namespace pwl
