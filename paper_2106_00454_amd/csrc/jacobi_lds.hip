// FP32 one-sided Jacobi with W resident in LDS (Sec. 3.1, H = C D C^T; Sec. 3.2
// step 2; Sec. 4.2, parallel cyclic-order Jacobi) for items with n <= 200.
//
// The method is the one-sided (Hestenes) Jacobi iteration on B = H + sigma I,
// with sigma from Gershgorin bounds so that B is positive definite: rotating
// the columns of W = B until they are mutually orthogonal gives W = B Q = Q L,
// so eigenvector m is w_m/|w_m| and its eigenvalue is |w_m| - sigma.  Only one
// n x n array is needed, which lets a 200 x 200 FP32 matrix live in the
// 160 KiB LDS of a gfx950 compute unit (two-sided Jacobi would need A and C).
// One work-group per item.  Output: eigenvalues (FP64 array, FP32 accuracy)
// and eigenvectors as a row-major FP32 workspace X[r*n + m], both sorted by
// ascending eigenvalue.
#include "jacobi_common.h"
#include "jacobi_quad.h"

namespace wpcd {
namespace {

template <int BLOCK, int G, int RMAX, int B>
__global__ __launch_bounds__(BLOCK) void jacobi_f32_lds_kernel(const ItemDev* __restrict__ items,
                                                               const int32_t* __restrict__ sel,
                                                               const GridDev* __restrict__ grids,
                                                               const double* __restrict__ v64,
                                                               float* __restrict__ x32, double* __restrict__ eval,
                                                               int32_t* __restrict__ status, int max_sweeps,
                                                               float tol, float stop, const int32_t* __restrict__ ref,
                                                               const double* __restrict__ work,
                                                               unsigned long long* counters) {
  extern __shared__ float W[];
  __shared__ int s_nrot;
  __shared__ float nrm[kMaxLdsN];
  constexpr bool kSorted = B == 0 || (B >= 5 && B <= 10);  // sorted columns, tracked norms
  constexpr bool kScaled = B >= 7 && B <= 10;               // scaled rotations
  constexpr int kPadCols = (B == 7 || B == 9 || B == 10) ? 2 : (B == 8 ? 4 : 1);  // W holds n rounded up to this many columns
  __shared__ float diag[kSorted ? kMaxLdsN : 1];
  __shared__ int perm[kSorted ? kMaxLdsN : 1];
  __shared__ float dsc[kScaled ? kMaxLdsN : 1];  // column scales of the scaled-rotation variants
  __shared__ int rot_flag[64];
  __shared__ float scratch[BLOCK / 64];
  __shared__ int bad;

  const int item = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  const ItemDev it = items[item];
  const int n = it.n, N = it.N;
  // variant 0 reads RMAX*G rows per column unguarded, variants 5 to 9 guard
  // only their last row chunk: the rows up to there (n .. rows-1) are zero
  const int rows = B == 0 ? max(n, RMAX * G) : ((B >= 5 && B <= 10) ? max(n, (RMAX - 1) * G) : n);
  const int ld = lds_stride(rows);
  const GridDev g = grids[it.grid];
  const double* V = v64 + it.v_off;
  for (int i = threadIdx.x; i < 64; i += BLOCK) rot_flag[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  // H = V + diag(e0) (V symmetric: row-major V is also column-major), rounded to FP32
  float sigma;
  if constexpr (kSorted) {
    // Variant 0 stores the columns of B = H + sigma I in descending order of
    // their norms (column j of W is column perm[j] of B; rows keep their
    // order, so each column is still an image of a basis vector): the
    // one-sided iteration then needs fewer sweeps (a NumPy model of the
    // coupled workload: 7.3 instead of 8.6 on average).  First pass over V:
    // Gershgorin bounds and |H e_c|^2, H_cc per column.
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    float lo = FLT_MAX, hi = -FLT_MAX;
    for (int c = grp; c < n; c += BLOCK / G) {
      float off = 0.f, h2 = 0.f, d = 0.f;
      for (int r = lane; r < n; r += G) {
        double h = V[c * n + r];
        if (r == c) h += g.e0[r % N];
        const float hf = (float)h;
        h2 = fmaf(hf, hf, h2);
        if (r == c) d = hf;
        else off += fabsf(hf);
      }
      off = group_sum<G>(off);
      h2 = group_sum<G>(h2);
      d = group_sum<G>(d);
      lo = fminf(lo, d - off);
      hi = fmaxf(hi, d + off);
      if (lane == 0) {
        nrm[c] = h2;
        diag[c] = d;
      }
    }
    lo = block_reduce<BLOCK>(lo, scratch, MinOp<float>());
    hi = block_reduce<BLOCK>(hi, scratch, MaxOp<float>());
    sigma = (lo < 0.f ? -lo : 0.f) + 0.05f * (hi - lo);
  }
  const int rid = (kSorted && ref) ? ref[item] : -1;
  if (rid >= 0) {
    // warm start from the reference item's eigenvectors Q0 (columns in
    // descending eigenvalue order, stored column-major as floats in the
    // reference's work-space): W = B Q0 = H Q0 + sigma Q0, with H Q0 formed
    // by the batched product into this item's x32 (column-major)
    const float* Y0 = x32 + it.v_off;
    const float* Q0 = reinterpret_cast<const float*>(work + items[rid].w_off);
    const int nr = n * rows;
    for (int e = threadIdx.x; e < nr; e += BLOCK) {
      const int j = e / rows, r = e - j * rows;
      W[j * ld + r] = r < n ? fmaf(sigma, Q0[j * n + r], Y0[j * n + r]) : 0.f;
    }
    if (kPadCols > 1)  // the zero columns completing the last block
      for (int e = threadIdx.x; e < (((n + kPadCols - 1) / kPadCols) * kPadCols - n) * rows; e += BLOCK)
        W[(n + e / rows) * ld + e % rows] = 0.f;
    __syncthreads();
  } else if constexpr (kSorted) {
    // |B e_c|^2 = |H e_c|^2 + 2 sigma H_cc + sigma^2; rank by descending norm.
    // A NaN key (NaN in V) ranks last: every comparison with NaN is false, so
    // without this two columns could take one rank and leave a slot of perm
    // unwritten; the item is flagged after the sweeps (its norms are NaN).
    for (int c = threadIdx.x; c < n; c += BLOCK) {
      const float key = nrm[c] + sigma * (2.f * diag[c] + sigma);
      diag[c] = key == key ? key : -INFINITY;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += BLOCK) {
      const float kc = diag[c];
      int rank = 0;
      for (int q = 0; q < n; ++q) rank += (diag[q] > kc || (diag[q] == kc && q < c)) ? 1 : 0;
      perm[rank] = c;
    }
    __syncthreads();
    const int nr = n * rows;
    for (int e = threadIdx.x; e < nr; e += BLOCK) {
      const int j = e / rows, r = e - j * rows;
      const int c = perm[j];
      double h = 0.0;
      if (r < n) {
        h = V[c * n + r];
        if (r == c) h += g.e0[r % N];
      }
      float w = (float)h;
      if (r == c) w += sigma;
      W[j * ld + r] = w;
    }
    if (kPadCols > 1)  // the zero columns completing the last block
      for (int e = threadIdx.x; e < (((n + kPadCols - 1) / kPadCols) * kPadCols - n) * rows; e += BLOCK)
        W[(n + e / rows) * ld + e % rows] = 0.f;
    __syncthreads();
  } else {
    const int nr = n * rows;
    for (int e = threadIdx.x; e < nr; e += BLOCK) {
      const int c = e / rows, r = e - c * rows;
      double h = 0.0;
      if (r < n) {
        h = V[c * n + r];
        if (r == c) h += g.e0[r % N];
      }
      W[c * ld + r] = (float)h;
    }
    __syncthreads();
    sigma = gershgorin_shift<float, BLOCK>(W, n, ld, scratch);
    for (int c = threadIdx.x; c < n; c += BLOCK) W[c * ld + c] += sigma;
    __syncthreads();
  }

  int sweeps;
  int nrot = 0;
  if (threadIdx.x == 0) s_nrot = 0;
  // (nrm holds |w|^2 during the sweeps of the tracked variants)
  if constexpr (B == 0)  // unblocked, tracked column norms
    sweeps = onesided_jacobi_lds_tracked<BLOCK, G, RMAX>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, nrot);
  else if constexpr (B == 5)  // blocks of 2 columns, tracked norms
    sweeps = onesided_jacobi_blocked_tracked<BLOCK, G, RMAX, 2>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, nrot);
  else if constexpr (B == 7)  // blocks of 2 columns, tracked norms, scaled rotations
    sweeps = onesided_jacobi_blocked_scaled<BLOCK, G, RMAX, 2>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, dsc,
                                                                nrot);
  else if constexpr (B == 10)  // as 7, halving ordering with one block kept in registers
    sweeps = onesided_jacobi_keep_scaled<BLOCK, G, RMAX>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, dsc, nrot);
  else if constexpr (B == 8)  // blocks of 4 columns, scaled rotations, one angle per quarter row
    sweeps = onesided_jacobi_parts<BLOCK, RMAX, 4>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, dsc, nrot);
  else if constexpr (B == 9)  // blocks of 2 columns, scaled rotations, one angle per half row
    sweeps = onesided_jacobi_parts<BLOCK, RMAX, 2>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, dsc, nrot);
  else if constexpr (B == 6)  // blocks of 4 columns, tracked norms
    sweeps = onesided_jacobi_blocked_tracked<BLOCK, G, RMAX, 4>(W, n, ld, tol, stop, max_sweeps, rot_flag, nrm, nrot);
  else  // unblocked, three dot products per pair
    sweeps = onesided_jacobi_lds<float, BLOCK, G, RMAX>(W, n, ld, tol, stop, max_sweeps, rot_flag);
  __syncthreads();

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
  if (counters) {  // work counters for the roofline: rotations, pair visits, sweeps
    if (nrot) atomicAdd(&s_nrot, nrot);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int sw = sweeps > max_sweeps ? max_sweeps : sweeps;
      atomicAdd(&counters[0], (unsigned long long)s_nrot);
      atomicAdd(&counters[1], (unsigned long long)sw * (unsigned long long)(n * (n - 1) / 2));
      atomicAdd(&counters[2], (unsigned long long)sw * (unsigned long long)n * (unsigned long long)n);
    }
  }
}

}  // namespace

hipError_t launch_jacobi_f32_lds(const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                 const GridDev* grids, const double* v64, float* x32, double* eval,
                                 int32_t* status, int max_sweeps, float tol, float stop, int block_cols,
                                 const int32_t* ref, const double* work, unsigned long long* counters,
                                 hipStream_t s) {
  if (max_n > kMaxLdsN) return hipErrorInvalidValue;
  if (max_sweeps > 64) return hipErrorInvalidValue;
  if (n_sel == 0) return hipSuccess;
  auto go = [&](auto kern, int block, int rows_min, int pad = 0) -> hipError_t {
    // pad: columns rounded up to a multiple of pad and 16 spare floats (scaled-rotation variants)
    const int cols = pad ? (max_n + pad - 1) / pad * pad : max_n;
    const size_t lds =
        ((size_t)lds_stride(max_n > rows_min ? max_n : rows_min) * cols + (pad ? 16 : 0)) * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_sel), dim3(block), lds, s, items, sel, grids, v64, x32, eval, status,
                       max_sweeps, tol, stop, ref, work, counters);
    return hipGetLastError();
  };
  // configuration value -> kernel variant: 0 (default) blocks of 2 columns
  // with tracked norms and scaled rotations in the halving ordering that
  // keeps one block per lane group in registers, 1 unblocked with three dot
  // products per pair, 2 unblocked with tracked norms, 3 blocks of 2 columns
  // with tracked norms and plain rotations, 4 blocks of 4 columns with
  // tracked norms, 5 blocks of 4 columns with scaled rotations and one angle
  // per quarter row, 6 blocks of 2 columns with one angle per half row
  // (jacobi_quad.h), 7 as 0 in the round-robin ordering
  static constexpr int kVariant[8] = {10, 1, 0, 5, 6, 8, 9, 7};
  if (block_cols < 0 || block_cols > 7) return hipErrorInvalidValue;
  const int B = kVariant[block_cols];
  if (max_n <= 64) {
    if (B == 0) return go(jacobi_f32_lds_kernel<256, 4, 16, 0>, 256, 64);
    if (B == 5) return go(jacobi_f32_lds_kernel<256, 16, 4, 5>, 256, 48);
    if (B == 7) return go(jacobi_f32_lds_kernel<256, 16, 4, 7>, 256, 48, 2);
    if (B == 10) return go(jacobi_f32_lds_kernel<256, 16, 4, 10>, 256, 48, 2);
    if (B == 8) return go(jacobi_f32_lds_kernel<128, 16, 4, 8>, 128, 48, 4);
    if (B == 9) return go(jacobi_f32_lds_kernel<256, 16, 4, 9>, 256, 48, 2);
    if (B == 6) return go(jacobi_f32_lds_kernel<256, 32, 2, 6>, 256, 32);
    if (B == 1) return go(jacobi_f32_lds_kernel<256, 4, 16, 1>, 256, 0);
    return hipErrorInvalidValue;
  }
  if (max_n <= 128) {
    if (B == 0) return go(jacobi_f32_lds_kernel<512, 8, 16, 0>, 512, 128);
    if (B == 5) return go(jacobi_f32_lds_kernel<512, 16, 8, 5>, 512, 112);
    if (B == 7) return go(jacobi_f32_lds_kernel<512, 16, 8, 7>, 512, 112, 2);
    if (B == 10) return go(jacobi_f32_lds_kernel<512, 16, 8, 10>, 512, 112, 2);
    if (B == 8) return go(jacobi_f32_lds_kernel<256, 16, 8, 8>, 256, 112, 4);
    if (B == 9) return go(jacobi_f32_lds_kernel<512, 16, 8, 9>, 512, 112, 2);
    if (B == 6) return go(jacobi_f32_lds_kernel<512, 32, 4, 6>, 512, 96);
    if (B == 1) return go(jacobi_f32_lds_kernel<512, 8, 16, 1>, 512, 0);
    return hipErrorInvalidValue;
  }
  if (B == 0) return go(jacobi_f32_lds_kernel<1024, 8, 25, 0>, 1024, 200);
  if (B == 5) return go(jacobi_f32_lds_kernel<1024, 16, 13, 5>, 1024, 192);
  if (B == 7) return go(jacobi_f32_lds_kernel<1024, 16, 13, 7>, 1024, 192, 2);
  if (B == 10) return go(jacobi_f32_lds_kernel<1024, 16, 13, 10>, 1024, 192, 2);
  if (B == 8) return go(jacobi_f32_lds_kernel<512, 16, 13, 8>, 512, 192, 4);
  if (B == 9) return go(jacobi_f32_lds_kernel<1024, 16, 13, 9>, 1024, 192, 2);
  if (B == 6) return go(jacobi_f32_lds_kernel<1024, 32, 7, 6>, 1024, 192);
  if (B == 1) return go(jacobi_f32_lds_kernel<1024, 8, 25, 1>, 1024, 0);
  return hipErrorInvalidValue;
}

}  // namespace wpcd
