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

// Generic kernel (items not taken by project8c_kernel).
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

// Tiled projection for ng = 8: one work-group per 32 x 32 tile of V in the
// upper block triangle (tile row <= tile column); a wavefront reads whole 16-byte-per-lane runs of one U row (64 lanes x 16 B =
// 1 KB contiguous per load for FP32): lane L of a pass holds E = 16/sizeof(T)
// consecutive elements of the 8-wide column block J = L / (8/E), forms their
// weighted partial sum, and the 8/E lanes of a block add theirs with DPP
// (quad_perm), so every 128-byte line of U is fetched by one load
// instruction.  Wavefront w takes the tile rows I0 + w, I0 + w + 4, ...; in a
// diagonal tile the lanes of blocks J < I issue no load.  Same arithmetic
// order for every element (weights applied per E-run, then per row), V
// written to (I, J) and (J, I) through the LDS tile.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
__global__ __launch_bounds__(256) void project8c_kernel(const ItemDev* __restrict__ items, int item0,
                                                        const GridDev* __restrict__ grids,
                                                        const T* __restrict__ u, double* __restrict__ v64) {
  constexpr int E = 16 / (int)sizeof(T);  // elements per lane and load
  constexpr int LB = 8 / E;               // lanes per 8-wide column block
  constexpr int JW = 64 / LB;             // column blocks per pass
  constexpr int NP = 32 / JW;             // passes per tile row
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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sub = lane % LB;  // which E-run of the block
  for (int pass = 0; pass < NP; ++pass) {
    const int jj = pass * JW + lane / LB;  // tile column of this lane
    const int J = J0 + jj;
    const bool colok = J < n;
    const int j = colok ? J % N : 0;
    T wb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) wb[e] = T(g.wk[j * 8 + sub * E + e]);
    const double sj = g.rsdk[j];
    // two tile rows (ii, ii + 4) per round: the 16 loads of a lane are all
    // issued before their sums; U is read once, so the loads do not keep it
    // in the caches (non-temporal)
    for (int i2 = w; i2 < 32; i2 += 8) {
      T x[2][8][E];
      bool needr[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ii = i2 + 4 * h, I = I0 + ii;
        needr[h] = I < n && colok && (ti < tj || ii <= jj);
        const T* up = u + it.u_off + (int64_t)(I < n ? I : 0) * 8 * M + (int64_t)J * 8 + sub * E;
#pragma unroll
        for (int al = 0; al < 8; ++al) {
          if (needr[h]) {
            if constexpr (E == 4) {
              const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(up + al * M));
#pragma unroll
              for (int e = 0; e < 4; ++e) x[h][al][e] = a[e];
            } else {
              const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(up + al * M));
              x[h][al][0] = a[0];
              x[h][al][1] = a[1];
            }
          } else {
#pragma unroll
            for (int e = 0; e < E; ++e) x[h][al][e] = T(0);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ii = i2 + 4 * h, I = I0 + ii;
        if (I >= n) break;  // wavefront-uniform
        const int i = I % N;
        T acc = T(0);
#pragma unroll
        for (int al = 0; al < 8; ++al) {
          T sm = T(0);
#pragma unroll
          for (int e = 0; e < E; ++e) sm = fma(wb[e], x[h][al][e], sm);
          // the block's runs: lanes L and L ^ 1 (and L ^ 2 for E = 2)
          if constexpr (sizeof(T) == 4) {
            sm += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sm), 0xB1, 0xF, 0xF, false));
          } else {
            const long long b = __double_as_longlong(sm);
            int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
            int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
            sm += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
            const long long b2 = __double_as_longlong(sm);
            lo = __builtin_amdgcn_update_dpp(0, (int)(b2 & 0xffffffffLL), 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, (int)(b2 >> 32), 0x4E, 0xF, 0xF, false);
            sm += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
          }
          acc = fma(T(g.wk[i * 8 + al]), sm, acc);
        }
        if (needr[h] && sub == 0) {
          const double v = (double)acc * g.rsdk[i] * sj;
          tile[ii][jj] = v;
          if (ti == tj) tile[jj][ii] = v;
        }
      }
    }
  }
  __syncthreads();
  double* V = v64 + it.v_off;
  const int cj = threadIdx.x & 31, r0 = threadIdx.x >> 5;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = r0 + 8 * r;
    if (I0 + rr < n && J0 + cj < n) V[(int64_t)(I0 + rr) * n + J0 + cj] = tile[rr][cj];
    if (ti < tj && J0 + rr < n && I0 + cj < n) V[(int64_t)(J0 + rr) * n + I0 + cj] = tile[cj][rr];
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
      hipLaunchKernelGGL(project8c_kernel<float>, dim3(gt, gy), dim3(bs), 0, s, items, i0, grids,
                         (const float*)u, v64);
      if (generic)
        hipLaunchKernelGGL(project_kernel<float>, dim3(gx, gy), dim3(bs), 0, s, items, i0, grids,
                           (const float*)u, v64);
    } else {
      hipLaunchKernelGGL(project8c_kernel<double>, dim3(gt, gy), dim3(bs), 0, s, items, i0, grids,
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
