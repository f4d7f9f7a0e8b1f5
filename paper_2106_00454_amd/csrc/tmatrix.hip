// On-shell T-matrix at every free-bin energy (Sec. 3.2, steps 3-5; App. B).
//
// One work-group per item:
//  1. classify the (ascending) eigenvalues: eps < 0 bound, eps > k_N^2 a
//     discrete state of the cut-off Hamiltonian, otherwise a scattering packet;
//     deal the scattering eigenvalues round-robin into n_ch families and build
//     each family's bins B_1 = 0, B_j = (e_{j-1} + e_j)/2,
//     B_{n+1} = e_n + (B_n - B_{n-1})/2 (Sec. 3.1);
//  2. for every free bin k (one wavefront per bin, lanes over eigenstates m)
//     evaluate the energy-averaged resolvent in FP64,
//       gbar_km = [F(b-c) - F(a-c) - F(b-d) + F(a-d) - i pi |[a,b]&[c,d]|]/((b-a)(d-c)),
//       F(x) = x ln|x|, free bin [a,b] = [k_{k-1}^2, k_k^2], packet bin [c,d],
//     or ln((b-eps)/(a-eps))/(b-a) for discrete states, and contract
//       T_ab(k) = V_(a,k),(b,k) + sum_m VC_(a,k),m VC_(b,k),m gbar_km
//     with VC_r,m = (eps_m - e_r) C_r,m, which equals (V C)_r,m for eigenpairs
//     of H0 + V because H0 is diagonal in the free packet basis.
// The resolvent table is always FP64 (its four x ln x terms cancel strongly for
// narrow low-energy bins).  The contraction is FP32 with FP32 accumulation in
// WPCD_MIXED mode and FP64 in WPCD_F64 mode.
#include "devutil.h"
#include "internal.h"

namespace wpcd {
namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double xlogx(double x) { return x == 0.0 ? 0.0 : x * log(fabs(x)); }

// Items with n <= 64 kMJ: each wavefront takes a contiguous run of bins, so
// the x ln x terms at the bins' upper boundary E_k carry over as the lower
// boundary terms of bin k + 1 (two logs per scattering pair instead of four;
// the same values, so the same result).  Lane l handles m = l + 64 j.
constexpr int kMJ = 4;
template <typename A, int K>
__device__ __forceinline__ void tmatrix_bins_carry(const ItemDev& it, const GridDev& g, const double* V,
                                                   const double* C, const double* eps, const double* lo,
                                                   const double* hi, int b0, int b1, double* t, int lane, int wave) {
  const int n = it.n, N = it.N;
  constexpr int NW = kBlock / 64;
  const int per = (N + NW - 1) / NW;
  const int k0 = wave * per, k1 = min(N, k0 + per);
  double fc[kMJ], fd[kMJ];  // F(E_k - c), F(E_k - d) at the current lower boundary
  if (k0 < k1) {
    const double a0 = g.eb[k0];
#pragma unroll
    for (int j = 0; j < kMJ; ++j) {
      const int m = lane + 64 * j;
      const bool sc = m < n && m >= b0 && m < b1;
      fc[j] = sc ? xlogx(a0 - lo[m]) : 0.0;
      fd[j] = sc ? xlogx(a0 - hi[m]) : 0.0;
    }
  }
  for (int k = k0; k < k1; ++k) {
    const double a = g.eb[k], b = g.eb[k + 1], de = b - a;
    const double ek = g.e0[k];
    A acc_re[K][K], acc_im[K][K];
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        acc_re[p][q] = A(0);
        acc_im[p][q] = A(0);
      }
#pragma unroll
    for (int j = 0; j < kMJ; ++j) {
      const int m = lane + 64 * j;
      if (m >= n) continue;
      const double em = eps[m];
      double gre, gim;
      if (m < b0 || m >= b1) {
        gre = log((b - em) / (a - em)) / de;
        gim = 0.0;
      } else {
        const double c = lo[m], d = hi[m];
        const double w = 1.0 / (de * (d - c));
        const double bc = xlogx(b - c), bd = xlogx(b - d);
        gre = (bc - fc[j] - bd + fd[j]) * w;
        fc[j] = bc;
        fd[j] = bd;
        const double ov = fmin(b, d) - fmax(a, c);
        gim = ov > 0.0 ? -kPi * ov * w : 0.0;
      }
      const double sh = em - ek;
      A vc[K];
#pragma unroll
      for (int q = 0; q < K; ++q) vc[q] = (A)(sh * C[(int64_t)(q * N + k) * n + m]);
      const A gr = (A)gre, gi = (A)gim;
#pragma unroll
      for (int p = 0; p < K; ++p)
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const A pr = vc[p] * vc[q];
          acc_re[p][q] = fma(pr, gr, acc_re[p][q]);
          acc_im[p][q] = fma(pr, gi, acc_im[p][q]);
        }
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const A sr = wave_total(acc_re[p][q]);
        const A si = wave_total(acc_im[p][q]);
        if (lane == 0) {
          const double vd = V[(int64_t)(p * N + k) * n + (q * N + k)];
          double* out = t + it.t_off + 2 * ((int64_t)(k * K + p) * K + q);
          out[0] = vd + (double)sr;
          out[1] = (double)si;
        }
      }
  }
}

// Items with n > 64 kMJ: wavefront w takes bins w, w + 4, ...; lanes over m.
template <typename A, int K>
__device__ __forceinline__ void tmatrix_bins(const ItemDev& it, const GridDev& g, const double* V, const double* C,
                                             const double* eps, const double* lo, const double* hi, int b0, int b1,
                                             double* t, int lane, int wave) {
  const int n = it.n, N = it.N;
  for (int k = wave; k < N; k += kBlock / 64) {
    const double a = g.eb[k], b = g.eb[k + 1], de = b - a;
    const double ek = g.e0[k];
    A acc_re[K][K], acc_im[K][K];
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        acc_re[p][q] = A(0);
        acc_im[p][q] = A(0);
      }
    for (int m = lane; m < n; m += 64) {
      const double em = eps[m];
      double gre, gim;
      if (m < b0 || m >= b1) {
        gre = log((b - em) / (a - em)) / de;
        gim = 0.0;
      } else {
        const double c = lo[m], d = hi[m];
        const double w = 1.0 / (de * (d - c));
        gre = (xlogx(b - c) - xlogx(a - c) - xlogx(b - d) + xlogx(a - d)) * w;
        const double ov = fmin(b, d) - fmax(a, c);
        gim = ov > 0.0 ? -kPi * ov * w : 0.0;
      }
      const double sh = em - ek;
      A vc[K];
#pragma unroll
      for (int q = 0; q < K; ++q) vc[q] = (A)(sh * C[(int64_t)(q * N + k) * n + m]);
      const A gr = (A)gre, gi = (A)gim;
#pragma unroll
      for (int p = 0; p < K; ++p)
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const A pr = vc[p] * vc[q];
          acc_re[p][q] = fma(pr, gr, acc_re[p][q]);
          acc_im[p][q] = fma(pr, gi, acc_im[p][q]);
        }
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const A sr = wave_total(acc_re[p][q]);
        const A si = wave_total(acc_im[p][q]);
        if (lane == 0) {
          const double vd = V[(int64_t)(p * N + k) * n + (q * N + k)];
          double* out = t + it.t_off + 2 * ((int64_t)(k * K + p) * K + q);
          out[0] = vd + (double)sr;
          out[1] = (double)si;
        }
      }
  }
}

template <typename A>
__global__ __launch_bounds__(kBlock) void tmatrix_kernel(const ItemDev* __restrict__ items,
                                                         const GridDev* __restrict__ grids,
                                                         const double* __restrict__ v64,
                                                         const double* __restrict__ eval,
                                                         const double* __restrict__ evec, double* __restrict__ t,
                                                         int32_t* __restrict__ status) {
  __shared__ double eps[kMaxN];
  __shared__ double lo[kMaxN];
  __shared__ double hi[kMaxN];
  __shared__ int s_bad, s_b0, s_b1;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n, N = it.N, K = it.nch;
  const GridDev g = grids[it.grid];
  const double etop = g.eb[N];
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_b0 = n;
    s_b1 = n;
  }
  __syncthreads();
  for (int m = threadIdx.x; m < n; m += kBlock) eps[m] = eval[it.e_off + m];
  __syncthreads();
  // b0 = number of bound states, b1 = first state above the free continuum
  for (int m = threadIdx.x; m < n; m += kBlock) {
    const double e = eps[m];
    if (!isfinite(e) || e == 0.0 || (m > 0 && e < eps[m - 1])) atomicOr(&s_bad, 1);
    if (e > 0.0 && (m == 0 || eps[m - 1] < 0.0)) s_b0 = m;
    if (e > etop && (m == 0 || eps[m - 1] <= etop)) s_b1 = m;
  }
  __syncthreads();
  const int b0 = s_b0 < s_b1 ? s_b0 : s_b1;
  const int b1 = s_b1;
  const int P = b1 - b0;
  if (P < 2 * K) {
    if (threadIdx.x == 0) s_bad = 1;
  }
  for (int m = threadIdx.x; m < n; m += kBlock) {
    if (m < b0 || m >= b1) {
      lo[m] = 0.0;
      hi[m] = 0.0;
      continue;
    }
    const int r = m - b0, kap = r % K, j = r / K;
    const int nk = (P - kap + K - 1) / K;
    if (nk < 2) continue;
    auto e_at = [&](int q) { return eps[b0 + kap + q * K]; };
    auto bnd = [&](int q) -> double {  // B_q of this family, q = 0..nk
      if (q == 0) return 0.0;
      if (q < nk) return 0.5 * (e_at(q - 1) + e_at(q));
      const double bm1 = 0.5 * (e_at(nk - 2) + e_at(nk - 1));
      const double bm2 = nk >= 3 ? 0.5 * (e_at(nk - 3) + e_at(nk - 2)) : 0.0;
      return e_at(nk - 1) + 0.5 * (bm1 - bm2);
    };
    lo[m] = bnd(j);
    hi[m] = bnd(j + 1);
    if (!(hi[m] > lo[m])) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  if (s_bad) {
    // flagged items get NaN T (so their phase shifts and cross sections are NaN too)
    double* tt = t + it.t_off;
    for (int e = threadIdx.x; e < 2 * N * K * K; e += kBlock) tt[e] = NAN;
    if (threadIdx.x == 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
    return;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* V = v64 + it.v_off;
  const double* C = evec + it.v_off;
  if (n <= 64 * kMJ) {
    if (K == 2)
      tmatrix_bins_carry<A, 2>(it, g, V, C, eps, lo, hi, b0, b1, t, lane, wave);
    else
      tmatrix_bins_carry<A, 1>(it, g, V, C, eps, lo, hi, b0, b1, t, lane, wave);
    if (threadIdx.x == 0) status[blockIdx.x] = 0;
    return;
  }
  if (K == 2)
    tmatrix_bins<A, 2>(it, g, V, C, eps, lo, hi, b0, b1, t, lane, wave);
  else
    tmatrix_bins<A, 1>(it, g, V, C, eps, lo, hi, b0, b1, t, lane, wave);
  if (threadIdx.x == 0) status[blockIdx.x] = 0;
}

}  // namespace

hipError_t launch_tmatrix(const ItemDev* items, int n_items, int max_n, const GridDev* grids, const double* v64,
                          const double* eval, const double* evec, int mode, double* t, int32_t* status,
                          hipStream_t s) {
  if (max_n > kMaxN) return hipErrorInvalidValue;
  if (mode == WPCD_MIXED)
    hipLaunchKernelGGL(tmatrix_kernel<float>, dim3(n_items), dim3(kBlock), 0, s, items, grids, v64, eval, evec, t,
                       status);
  else
    hipLaunchKernelGGL(tmatrix_kernel<double>, dim3(n_items), dim3(kBlock), 0, s, items, grids, v64, eval, evec, t,
                       status);
  return hipGetLastError();
}

}  // namespace wpcd
