// Potential projection onto momentum wave packets (Sec. 3.2, the packet
// potential matrix as a double integral over two bins, here by the per-bin
// Gauss rule):
//   V_(a,i),(b,j) = (dk_i dk_j)^(-1/2) sum_{alpha in i} sum_{beta in j}
//                   (w k)_alpha (w k)_beta U_(a,alpha),(b,beta).
// U is symmetric, so only its upper block triangle is read: one thread
// produces V_IJ for I <= J from an ng x ng block of U and writes it to both
// (I,J) and (J,I), which keeps V exactly symmetric whatever the summation order.
// Every U element of the upper triangle is read once: the kernel is HBM-bound.
// A wavefront covers 64 consecutive V columns, i.e. 64*ng consecutive U columns
// of ng rows, so each thread issues contiguous loads of its ng-wide segments.
#include "internal.h"

namespace wpcd {
namespace {

template <typename T, int NG>
__device__ __forceinline__ T block_sum(const T* __restrict__ up, int64_t ld, const double* __restrict__ wa,
                                       const double* __restrict__ wb) {
  T acc = T(0);
#pragma unroll
  for (int al = 0; al < NG; ++al) {
    const T* row = up + al * ld;
    T s = T(0);
#pragma unroll
    for (int be = 0; be < NG; ++be) s = fma(T(wb[be]), row[be], s);
    acc = fma(T(wa[al]), s, acc);
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ T block_sum_rt(const T* __restrict__ up, int64_t ld, const double* __restrict__ wa,
                                          const double* __restrict__ wb, int ng) {
  T acc = T(0);
  for (int al = 0; al < ng; ++al) {
    const T* row = up + al * ld;
    T s = T(0);
    for (int be = 0; be < ng; ++be) s = fma(T(wb[be]), row[be], s);
    acc = fma(T(wa[al]), s, acc);
  }
  return acc;
}

// grid: x = blocks over the item's n*n elements, y = item (chunked by the host)
template <typename T>
__global__ __launch_bounds__(256) void project_kernel(const ItemDev* __restrict__ items, int item0,
                                                      const GridDev* __restrict__ grids,
                                                      const T* __restrict__ u, double* __restrict__ v64) {
  const ItemDev it = items[item0 + blockIdx.y];
  if (it.basis >= 0) return;  // projected from a resident basis instead
  const int n = it.n;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int I = (int)(e / n), J = (int)(e - (int64_t)I * n);
  if (I > J) return;
  const GridDev g = grids[it.grid];
  const int N = it.N, ng = it.ng;
  const int i = I % N, j = J % N;
  const int64_t M = (int64_t)n * ng;
  const T* up = u + it.u_off + (int64_t)I * ng * M + (int64_t)J * ng;
  const double* wa = g.wk + (int64_t)i * ng;
  const double* wb = g.wk + (int64_t)j * ng;
  T acc;
  if (ng == 8)
    acc = block_sum<T, 8>(up, M, wa, wb);
  else if (ng == 4)
    acc = block_sum<T, 4>(up, M, wa, wb);
  else
    acc = block_sum_rt<T>(up, M, wa, wb, ng);
  const double v = (double)acc * g.rsdk[i] * g.rsdk[j];
  v64[it.v_off + e] = v;
  v64[it.v_off + (int64_t)J * n + I] = v;
}

// Affine potentials (the projection is linear in U): V = sum_t c_t B_t over
// the item's resident basis, one thread per element of V, FP64 throughout.
// Every B_t is exactly symmetric and the sum runs in the same order for (I,J)
// and (J,I), so V is exactly symmetric.
__global__ __launch_bounds__(256) void project_affine_kernel(const ItemDev* __restrict__ items, int item0,
                                                             const BasisDev* __restrict__ bases,
                                                             const double* __restrict__ coef,
                                                             double* __restrict__ v64) {
  const ItemDev it = items[item0 + blockIdx.y];
  if (it.basis < 0) return;
  const int64_t nn = (int64_t)it.n * it.n;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const BasisDev bs = bases[it.basis];
  const double* c = coef + it.c_off;
  double acc = 0.0;
  for (int t = 0; t < bs.n_terms; ++t) acc = fma(c[t], bs.b[t * nn + e], acc);
  v64[it.v_off + e] = acc;
}

}  // namespace

hipError_t launch_project_affine(const ItemDev* items, int n_items, int max_n, const BasisDev* bases,
                                 const double* coef, double* v64, hipStream_t s) {
  const int bs = 256;
  const unsigned gx = (unsigned)(((int64_t)max_n * max_n + bs - 1) / bs);
  for (int i0 = 0; i0 < n_items; i0 += 65535) {
    const unsigned gy = (unsigned)((n_items - i0) < 65535 ? (n_items - i0) : 65535);
    hipLaunchKernelGGL(project_affine_kernel, dim3(gx, gy), dim3(bs), 0, s, items, i0, bases, coef, v64);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_project(const ItemDev* items, int n_items, int max_n, const GridDev* grids, const void* u,
                          int u_dtype, double* v64, hipStream_t s) {
  const int bs = 256;
  const unsigned gx = (unsigned)(((int64_t)max_n * max_n + bs - 1) / bs);
  for (int i0 = 0; i0 < n_items; i0 += 65535) {
    const unsigned gy = (unsigned)((n_items - i0) < 65535 ? (n_items - i0) : 65535);
    if (u_dtype == WPCD_DTYPE_F32)
      hipLaunchKernelGGL(project_kernel<float>, dim3(gx, gy), dim3(bs), 0, s, items, i0, grids,
                         (const float*)u, v64);
    else
      hipLaunchKernelGGL(project_kernel<double>, dim3(gx, gy), dim3(bs), 0, s, items, i0, grids,
                         (const double*)u, v64);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace wpcd
