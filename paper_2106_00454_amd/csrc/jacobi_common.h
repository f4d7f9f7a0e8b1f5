// Helpers shared by the two eigensolver sources (LDS and device-memory Jacobi).
#pragma once

#include <float.h>

#include "devutil.h"
#include "internal.h"

namespace wpcd {

template <typename T>
struct MinOp {
  __device__ T operator()(T a, T b) const { return a < b ? a : b; }
};
template <typename T>
struct MaxOp {
  __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};

// Gershgorin interval of the symmetric matrix stored column-major in W
// (column sums equal row sums).  Returns the shift sigma = max(0, -lo) + 0.05 (hi - lo).
template <typename T, int BLOCK>
__device__ T gershgorin_shift(const T* W, int n, int ld, T* scratch) {
  T lo = T(FLT_MAX), hi = T(-FLT_MAX);
  for (int c = threadIdx.x; c < n; c += BLOCK) {
    const T* col = W + (int64_t)c * ld;
    T s = T(0);
    for (int r = 0; r < n; ++r) s += (r == c) ? T(0) : fabs(col[r]);
    const T d = col[c];
    lo = d - s < lo ? d - s : lo;
    hi = d + s > hi ? d + s : hi;
  }
  lo = block_reduce<BLOCK>(lo, scratch, MinOp<T>());
  hi = block_reduce<BLOCK>(hi, scratch, MaxOp<T>());
  const T base = lo < T(0) ? -lo : T(0);
  return base + T(0.05) * (hi - lo);
}

// Column stride of W in LDS: the smallest ld >= n with ld = 8 (mod 64).  In a
// round-robin step the 8 lane groups of a wavefront read 8 consecutive columns
// (rows lane + 8t), so column starts 8 banks apart make the 8 groups cover 64
// distinct banks: conflict-free on 64 banks, the minimal two passes on 32.
__host__ __device__ constexpr int lds_stride(int n) { return n + ((8 - n) % 64 + 64) % 64; }

}  // namespace wpcd
