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

// Generic kernel (items not taken by project8_kernel).
// grid: x = blocks over the item's n*n elements, y = item (chunked by the host)
template <typename T>
__global__ __launch_bounds__(256) void project_kernel(const ItemDev* __restrict__ items, int item0,
                                                      const GridDev* __restrict__ grids,
                                                      const T* __restrict__ u, double* __restrict__ v64) {
  const ItemDev it = items[item0 + blockIdx.y];
  if (it.basis >= 0 || project_tiled(it, u, (int)sizeof(T))) return;  // resident basis / tiled kernel
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

// 8 consecutive U elements of one row (two 16-byte loads)
__device__ __forceinline__ void load8(const float* p, float (&x)[8]) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
  x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}
__device__ __forceinline__ void load8(const double* p, double (&x)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double2 a = reinterpret_cast<const double2*>(p)[q];
    x[2 * q] = a.x;
    x[2 * q + 1] = a.y;
  }
}

// Tiled projection for ng = 8: one work-group per 32 x 32 tile of V in the
// upper block triangle (tile row <= tile column).  Thread t produces
// V[I0 + t/32 + 8r][J0 + t%32], r = 0..3, each from an 8 x 8 block of U
// (8 rows of 8 consecutive elements: a wavefront reads 32 consecutive
// 32-byte segments of each of two U rows).  Inside a diagonal tile only
// I <= J is computed and mirrored, so V is exactly symmetric.  The tile is
// staged in LDS and written to (I, J) and, transposed, to (J, I) as rows of
// 32 consecutive doubles.  Taken by items whose U block starts on a 16-byte
// boundary (the 16-byte loads stay aligned: rows are 8n elements long).
// grid: x = upper tiles of the largest item, y = item (chunked by the host)
template <typename T>
__global__ __launch_bounds__(256) void project8_kernel(const ItemDev* __restrict__ items, int item0,
                                                       const GridDev* __restrict__ grids,
                                                       const T* __restrict__ u, double* __restrict__ v64) {
  __shared__ double tile[32][33];
  const ItemDev it = items[item0 + blockIdx.y];
  if (it.basis >= 0 || !project_tiled(it, u, (int)sizeof(T))) return;
  const int n = it.n;
  const int nt = (n + 31) / 32;
  int t = blockIdx.x, ti = 0;
  while (ti < nt && t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  if (ti >= nt) return;
  const int tj = ti + t;
  const int I0 = ti * 32, J0 = tj * 32;
  const GridDev g = grids[it.grid];
  const int N = it.N;
  const int64_t M = (int64_t)n * 8;
  const int jj = threadIdx.x & 31, ii0 = threadIdx.x >> 5;
  const int J = J0 + jj;
  double wb[8];
  double sj = 0.0;
  if (J < n) {
    const int j = J % N;
#pragma unroll
    for (int b = 0; b < 8; ++b) wb[b] = g.wk[j * 8 + b];
    sj = g.rsdk[j];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = ii0 + 8 * r, I = I0 + ii;
    if (I < n && J < n && (ti < tj || ii <= jj)) {
      const int i = I % N;
      const T* up = u + it.u_off + (int64_t)I * 8 * M + (int64_t)J * 8;
      T acc = T(0);
#pragma unroll
      for (int al = 0; al < 8; ++al) {
        T x[8];
        load8(up + al * M, x);
        T s = T(0);
#pragma unroll
        for (int b = 0; b < 8; ++b) s = fma(T(wb[b]), x[b], s);
        acc = fma(T(g.wk[i * 8 + al]), s, acc);
      }
      const double v = (double)acc * g.rsdk[i] * sj;
      tile[ii][jj] = v;
      if (ti == tj) tile[jj][ii] = v;
    }
  }
  __syncthreads();
  double* V = v64 + it.v_off;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = ii0 + 8 * r;
    if (I0 + rr < n && J0 + jj < n) V[(int64_t)(I0 + rr) * n + J0 + jj] = tile[rr][jj];
    if (ti < tj && J0 + rr < n && I0 + jj < n) V[(int64_t)(J0 + rr) * n + I0 + jj] = tile[jj][rr];
  }
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
                          int u_dtype, double* v64, bool generic, hipStream_t s) {
  const int bs = 256;
  const unsigned gx = (unsigned)(((int64_t)max_n * max_n + bs - 1) / bs);
  const int nt = (max_n + 31) / 32;
  const unsigned gt = (unsigned)(nt * (nt + 1) / 2);
  for (int i0 = 0; i0 < n_items; i0 += 65535) {
    const unsigned gy = (unsigned)((n_items - i0) < 65535 ? (n_items - i0) : 65535);
    if (u_dtype == WPCD_DTYPE_F32) {
      hipLaunchKernelGGL(project8_kernel<float>, dim3(gt, gy), dim3(bs), 0, s, items, i0, grids,
                         (const float*)u, v64);
      if (generic)
        hipLaunchKernelGGL(project_kernel<float>, dim3(gx, gy), dim3(bs), 0, s, items, i0, grids,
                           (const float*)u, v64);
    } else {
      hipLaunchKernelGGL(project8_kernel<double>, dim3(gt, gy), dim3(bs), 0, s, items, i0, grids,
                         (const double*)u, v64);
      if (generic)
        hipLaunchKernelGGL(project_kernel<double>, dim3(gx, gy), dim3(bs), 0, s, items, i0, grids,
                           (const double*)u, v64);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace wpcd
