// Eigensolvers of H = H0 + V in the free wave-packet basis (Sec. 3.1,
// H = C D C^T; Sec. 3.2 step 2; Sec. 4.2, parallel cyclic-order Jacobi).
//
// The method is the one-sided (Hestenes) Jacobi iteration on B = H + sigma I,
// with sigma from Gershgorin bounds so that B is positive definite: rotating
// the columns of W = B until they are mutually orthogonal gives W = B Q = Q L,
// so eigenvector m is w_m/|w_m| and its eigenvalue is |w_m| - sigma.  Only one
// n x n array is needed, which lets a 200 x 200 FP32 matrix live in the
// 160 KiB LDS of a gfx950 compute unit (two-sided Jacobi would need A and C).
//
//  * jacobi_f32_lds_kernel: one work-group per item, W in LDS, FP32.  Output:
//    eigenvalues (FP64 array, FP32 accuracy) and eigenvectors as a row-major
//    FP32 workspace X[r*n + m], both sorted by ascending eigenvalue.
//  * jacobi_global_kernel: same iteration with W in device memory (any n), in
//    FP64 for the plain path (output straight to the caller's arrays) or in
//    FP32 for mixed-path items too large for LDS (output as above).
#include <float.h>

#include "devutil.h"
#include "internal.h"

namespace wpcd {
namespace {

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

template <int BLOCK, int G, int RMAX, int B>
__global__ __launch_bounds__(BLOCK) void jacobi_f32_lds_kernel(const ItemDev* __restrict__ items,
                                                               const int32_t* __restrict__ sel,
                                                               const GridDev* __restrict__ grids,
                                                               const double* __restrict__ v64,
                                                               float* __restrict__ x32, double* __restrict__ eval,
                                                               int32_t* __restrict__ status, int max_sweeps,
                                                               float tol) {
  extern __shared__ float W[];
  __shared__ float nrm[kMaxLdsN];
  __shared__ int rot_flag[64];
  __shared__ float scratch[BLOCK / 64];
  __shared__ int bad;

  const int item = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  const ItemDev it = items[item];
  const int n = it.n, N = it.N;
  const int ld = lds_stride(n);
  const GridDev g = grids[it.grid];
  const double* V = v64 + it.v_off;
  for (int i = threadIdx.x; i < 64; i += BLOCK) rot_flag[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  // H = V + diag(e0) (V symmetric: row-major V is also column-major), rounded to FP32
  const int nn = n * n;
  for (int e = threadIdx.x; e < nn; e += BLOCK) {
    const int c = e / n, r = e - c * n;
    double h = V[e];
    if (r == c) h += g.e0[r % N];
    W[c * ld + r] = (float)h;
  }
  __syncthreads();
  const float sigma = gershgorin_shift<float, BLOCK>(W, n, ld, scratch);
  for (int c = threadIdx.x; c < n; c += BLOCK) W[c * ld + c] += sigma;
  __syncthreads();

  const int sweeps = onesided_jacobi_blocked<float, BLOCK, G, RMAX, B>(W, n, ld, tol, max_sweeps, rot_flag);

  // column norms
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  for (int c = grp; c < n; c += ngrp) {
    const float* col = W + c * ld;
    float s2 = 0.f;
    for (int r = lane; r < n; r += G) s2 = fmaf(col[r], col[r], s2);
    s2 = group_sum<G>(s2);
    if (lane == 0) nrm[c] = sqrtf(s2);
  }
  __syncthreads();
  // rank sort (ties by index), eigenvalue |w| - sigma, eigenvector w/|w|
  float* X = x32 + it.v_off;
  double* ev = eval + it.e_off;
  for (int c = grp; c < n; c += ngrp) {
    const float nc = nrm[c];
    float cnt = 0.f;
    for (int i = lane; i < n; i += G) {
      const float ni = nrm[i];
      cnt += (ni < nc || (ni == nc && i < c)) ? 1.f : 0.f;
    }
    const int rank = (int)group_sum<G>(cnt);
    if (!(nc > 0.f) || !isfinite(nc)) {
      if (lane == 0) bad = 1;
      continue;
    }
    if (lane == 0) ev[rank] = (double)nc - (double)sigma;
    // divide (not multiply by 1/|w|): a column that never rotated becomes an exact unit vector
    const float* col = W + c * ld;
    for (int r = lane; r < n; r += G) X[(int64_t)r * n + rank] = col[r] / nc;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    status[item] = bad ? WPCD_ERR_NUMERIC : (sweeps > max_sweeps ? WPCD_ERR_NOCONV : sweeps);
}

// ---------------------------------------------------------- device-memory path
// W (n x n, column-major) lives in the item's device work-space; every pair
// step reads its two columns twice (Gram entries, then rotation) through the
// caches.  T = double: the plain FP64 path, eigenvalues as Rayleigh quotients
// v^T H v / v^T v of v = w/|w| (exact for a diagonal H, free of the shift's
// rounding), eigenvectors written straight to the caller's FP64 array.
// T = float: the mixed path for items too large for LDS; eigenvalues |w| - sigma
// and FP32 eigenvectors in the row-major work-space x32, as the LDS kernel.
template <typename T, int BLOCK, int G>
__global__ __launch_bounds__(BLOCK) void jacobi_global_kernel(const ItemDev* __restrict__ items,
                                                              const int32_t* __restrict__ sel,
                                                              const GridDev* __restrict__ grids,
                                                              const double* __restrict__ v64, double* work,
                                                              double* __restrict__ evec, float* __restrict__ x32,
                                                              double* __restrict__ eval,
                                                              int32_t* __restrict__ status, int max_sweeps, T tol) {
  __shared__ int rot_flag[64];
  __shared__ T scratch[BLOCK / 64];
  __shared__ int bad;
  __shared__ int rank_of[kMaxN];
  __shared__ double rq[kMaxN];
  __shared__ double nrm[kMaxN];
  const int item = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  const ItemDev it = items[item];
  const int n = it.n, N = it.N;
  const int ld = n;
  const GridDev g = grids[it.grid];
  const double* V = v64 + it.v_off;
  T* W = reinterpret_cast<T*>(work + it.w_off);
  for (int i = threadIdx.x; i < 64; i += BLOCK) rot_flag[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += BLOCK) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    double h = V[e];
    if (r == c) h += g.e0[r % N];
    W[e] = (T)h;
  }
  __syncthreads();
  const T sigma = gershgorin_shift<T, BLOCK>(W, n, ld, scratch);
  for (int c = threadIdx.x; c < n; c += BLOCK) W[(int64_t)c * ld + c] += sigma;
  __syncthreads();

  const int npair = (n + 1) >> 1, ne = npair << 1;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  int sweeps = max_sweeps + 1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int step = 0; step < ne - 1; ++step) {
      for (int pr = grp; pr < npair; pr += ngrp) {
        const int p = rr_index(pr, step, ne), q = rr_index(ne - 1 - pr, step, ne);
        if (p >= n || q >= n) continue;
        T* wp = W + (int64_t)p * ld;
        T* wq = W + (int64_t)q * ld;
        T al = 0, be = 0, ga = 0;
        for (int r = lane; r < n; r += G) {
          const T a = wp[r], b = wq[r];
          al = fma(a, a, al);
          be = fma(b, b, be);
          ga = fma(a, b, ga);
        }
        al = group_sum<G>(al);
        be = group_sum<G>(be);
        ga = group_sum<G>(ga);
        const T nab = sqrt(al * be);
        if (fabs(ga) > tol * nab) {
          T c, s;
          hestenes_rotation(al, be, ga, c, s);
          for (int r = lane; r < n; r += G) {
            const T a = wp[r], b = wq[r];
            wp[r] = c * a - s * b;
            wq[r] = s * a + c * b;
          }
          if (lane == 0) atomicMax(&rot_flag[sweep], __float_as_int((float)(fabs(ga) / nab)));
        }
      }
      __syncthreads();
    }
    if (__int_as_float(rot_flag[sweep]) < 8.0f * (float)tol) {
      sweeps = sweep + 1;
      break;
    }
  }
  // column norms and eigenvalue estimates
  for (int c = grp; c < n; c += ngrp) {
    const T* col = W + (int64_t)c * ld;
    T s2 = 0;
    for (int r = lane; r < n; r += G) s2 = fma(col[r], col[r], s2);
    const T nc = sqrt(group_sum<G>(s2));
    double lam = (double)nc - (double)sigma;
    if (sizeof(T) == 8) {
      // v = w/|w| by division, so an unrotated column is an exact unit vector
      double q = 0, vv = 0;
      for (int r = lane; r < n; r += G) {
        const double* hrow = V + (int64_t)r * n;
        double hv = 0;
        for (int t = 0; t < n; ++t) hv = fma(hrow[t], (double)col[t] / (double)nc, hv);
        const double vr = (double)col[r] / (double)nc;
        hv = fma(g.e0[r % N], vr, hv);
        q = fma(vr, hv, q);
        vv = fma(vr, vr, vv);
      }
      q = group_sum<G>(q);
      vv = group_sum<G>(vv);
      lam = q / vv;
    }
    if (lane == 0) {
      nrm[c] = (double)nc;
      rq[c] = lam;
    }
  }
  __syncthreads();
  for (int c = grp; c < n; c += ngrp) {
    const double lc = rq[c];
    double cnt = 0;
    for (int i = lane; i < n; i += G) {
      const double li = rq[i];
      cnt += (li < lc || (li == lc && i < c)) ? 1.0 : 0.0;
    }
    cnt = group_sum<G>(cnt);
    if (lane == 0) rank_of[c] = (int)cnt;
  }
  __syncthreads();
  for (int c = grp; c < n; c += ngrp) {
    const double nc = nrm[c];
    if (!(nc > 0.0) || !isfinite(nc) || !isfinite(rq[c])) {
      if (lane == 0) bad = 1;
      continue;
    }
    const int rank = rank_of[c];
    const T* col = W + (int64_t)c * ld;
    if (sizeof(T) == 8) {
      double* X = evec + it.v_off;
      for (int r = lane; r < n; r += G) X[(int64_t)r * n + rank] = (double)col[r] / nc;
    } else {
      float* X = x32 + it.v_off;
      for (int r = lane; r < n; r += G) X[(int64_t)r * n + rank] = (float)col[r] / (float)nc;
    }
  }
  __syncthreads();
  double* ev = eval + it.e_off;
  for (int c = threadIdx.x; c < n; c += BLOCK) ev[rank_of[c]] = rq[c];
  if (threadIdx.x == 0)
    status[item] = bad ? WPCD_ERR_NUMERIC : (sweeps > max_sweeps ? WPCD_ERR_NOCONV : sweeps);
}

}  // namespace

hipError_t launch_jacobi_f32_lds(const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                 const GridDev* grids, const double* v64, float* x32, double* eval,
                                 int32_t* status, int max_sweeps, float tol, int block_cols, hipStream_t s) {
  if (max_n > kMaxLdsN) return hipErrorInvalidValue;
  if (max_sweeps > 64) return hipErrorInvalidValue;
  if (n_sel == 0) return hipSuccess;
  const int ld = lds_stride(max_n);
  const size_t lds = (size_t)ld * max_n * sizeof(float);
  auto go = [&](auto kern, int block) -> hipError_t {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_sel), dim3(block), lds, s, items, sel, grids, v64, x32, eval, status,
                       max_sweeps, tol);
    return hipGetLastError();
  };
  // column block width: 0 picks the default per size class
  const int B = block_cols != 0 ? block_cols : 1;
  if (max_n <= 64) {
    if (B == 1) return go(jacobi_f32_lds_kernel<256, 4, 16, 1>, 256);
    if (B == 2) return go(jacobi_f32_lds_kernel<256, 16, 4, 2>, 256);
    return go(jacobi_f32_lds_kernel<128, 16, 4, 4>, 128);
  }
  if (max_n <= 128) {
    if (B == 1) return go(jacobi_f32_lds_kernel<512, 8, 16, 1>, 512);
    if (B == 2) return go(jacobi_f32_lds_kernel<512, 16, 8, 2>, 512);
    return go(jacobi_f32_lds_kernel<256, 16, 8, 4>, 256);
  }
  if (B == 1) return go(jacobi_f32_lds_kernel<1024, 8, 25, 1>, 1024);
  if (B == 2) return go(jacobi_f32_lds_kernel<1024, 16, 13, 2>, 1024);
  return go(jacobi_f32_lds_kernel<512, 16, 13, 4>, 512);
}

hipError_t launch_jacobi_global(int mixed, const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                const GridDev* grids, const double* v64, double* work, double* evec, float* x32,
                                double* eval, int32_t* status, int max_sweeps, double tol, hipStream_t s) {
  if (max_n > kMaxN || max_sweeps > 64) return hipErrorInvalidValue;
  if (n_sel == 0) return hipSuccess;
  if (mixed)
    hipLaunchKernelGGL((jacobi_global_kernel<float, 1024, 8>), dim3(n_sel), dim3(1024), 0, s, items, sel, grids, v64,
                       work, evec, x32, eval, status, max_sweeps, (float)tol);
  else
    hipLaunchKernelGGL((jacobi_global_kernel<double, 1024, 8>), dim3(n_sel), dim3(1024), 0, s, items, sel, grids,
                       v64, work, evec, x32, eval, status, max_sweeps, tol);
  return hipGetLastError();
}

}  // namespace wpcd
