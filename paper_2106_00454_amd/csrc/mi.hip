// Matrix-inversion (MI) solution of the partial-wave LS equation (Sec. 2.1,
// the wave-matrix form of the discretised LS equation and its K-matrix
// variant; Sec. 4.1, one LU factorisation per energy), batched over
// (item, energy): the comparison method of the paper, on the same device.
//
// For on-shell momentum p, N_Q Gauss-Legendre nodes q_j (weights w_j) on
// [0, L] and the on-shell point appended as node N_Q, the principal-value
// discretisation of the K-matrix equation
//   K(q', q) = U(q', q) + PV int_0^L dk k^2 U(q', k) K(k, q)/(p^2 - k^2)
// reads (1 - U diag(D)) K = U with
//   D_j = w_j q_j^2/(p^2 - q_j^2)                                  (j < N_Q),
//   D_NQ = -p^2 sum_j w_j/(p^2 - q_j^2) + (p/2) ln((L + p)/(L - p)),
// the subtraction term of the pole with the cut-off's principal-value log.
// Coupled items (n_ch = 2) stack both orbital channels channel-major, so the
// system has m = n_ch (N_Q + 1) unknowns per right-hand side, and the
// on-shell columns b = 0..n_ch-1 give the n_ch x n_ch on-shell K_ab(p).
//
// One work-group per (energy, item): the augmented matrix [1 - U D | U_on]
// in LDS (FP64, m (m + n_ch) doubles), Gaussian elimination with partial
// pivoting by rows.  The unknowns are ordered with the on-shell ones last,
// so after the elimination they follow from the trailing n_ch x n_ch
// triangle without a back substitution.  Then S = (1 - i pi p K/2)(1 + i pi
// p K/2)^-1 (exactly unitary for real symmetric K), the phase shifts, the
// Stapp mixing angle and the item's term (2J+1) sum_a (1 - Re S_aa) of the
// total cross section at p (App. A), summed per sample by a second kernel.
#include <float.h>

#include "internal.h"

namespace wpcd {
namespace {

constexpr int kMiBlock = 256;
constexpr double kPi = 3.14159265358979323846;
constexpr double kRadToDeg = 57.295779513082320876798;

__device__ __forceinline__ double wave_max_abs_arg(double v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  return v;
}

// Unknown / row index r of the system -> (channel a, mesh point i): the
// first n_ch N_Q rows are the quadrature nodes of channel a = r / N_Q, the
// last n_ch the on-shell points of channel a = r - n_ch N_Q.
__device__ __forceinline__ void mi_unknown(int r, int nq, int K, int& a, int& i) {
  if (r < K * nq) {
    a = r / nq;
    i = r - a * nq;
  } else {
    a = r - K * nq;
    i = nq;
  }
}

__global__ __launch_bounds__(kMiBlock) void mi_solve_kernel(const MiItemDev* __restrict__ items, int nq, int ne,
                                                            const double* __restrict__ qw,
                                                            const double* __restrict__ pts, double cutoff,
                                                            const double* __restrict__ u, double* __restrict__ kmat,
                                                            double* __restrict__ delta, double* __restrict__ mix,
                                                            double* __restrict__ loss, int32_t* __restrict__ status) {
  extern __shared__ double A[];
  __shared__ double Dv[kMaxMiNq + 1];
  __shared__ double red[kMiBlock / 64];
  __shared__ int redi[kMiBlock / 64];
  __shared__ int s_piv, s_bad;
  const int e = blockIdx.x;
  const int item = blockIdx.y;
  const MiItemDev it = items[item];
  const int K = it.nch;
  const int m = K * (nq + 1);
  const int ld = m + K;  // augmented row: m coefficients, K right-hand sides
  const int P = nq + ne;
  const double p = pts[nq + e];
  const double p2 = p * p;
  // D vector (FP64): quadrature part and the pole-subtraction term
  double part = 0.0;
  for (int j = threadIdx.x; j < nq; j += kMiBlock) {
    const double q = pts[j], w = qw[j];
    const double den = p2 - q * q;
    Dv[j] = w * q * q / den;
    part += w / den;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kMiBlock / 64; ++w) s += red[w];
    Dv[nq] = -p2 * s + 0.5 * p * log((cutoff + p) / (cutoff - p));
  }
  __syncthreads();
  // [1 - U D | U(:, on-shell)]: U of the item on the point set (n_ch P)^2,
  // channel-major; mesh point i of the system is point i of the set for
  // i < N_Q and point N_Q + e (this energy's p) for i = N_Q
  const double* U = u + it.u_off;
  const int64_t lu = (int64_t)K * P;
  for (int idx = threadIdx.x; idx < m * ld; idx += kMiBlock) {
    const int r = idx / ld, c = idx - r * ld;
    int a, i;
    mi_unknown(r, nq, K, a, i);
    const int ri = a * P + (i < nq ? i : nq + e);
    double v;
    if (c < m) {
      int b, j;
      mi_unknown(c, nq, K, b, j);
      const int cj = b * P + (j < nq ? j : nq + e);
      v = (r == c ? 1.0 : 0.0) - U[ri * lu + cj] * Dv[j];
    } else {
      const int b = c - m;
      v = U[ri * lu + b * P + nq + e];
    }
    A[idx] = v;
  }
  __syncthreads();
  // Gaussian elimination with partial pivoting (rows) down to the trailing
  // K x K block of the on-shell unknowns
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < m - 1; ++k) {
    double best = -1.0;
    int bi = m;
    for (int i = k + threadIdx.x; i < m; i += kMiBlock) {
      const double v = fabs(A[i * ld + k]);
      if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
      }
    }
    best = wave_max_abs_arg(best, bi);
    if (lane == 0) {
      red[wave] = best;
      redi[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = red[0];
      int bx = redi[0];
      for (int w = 1; w < kMiBlock / 64; ++w)
        if (red[w] > bv || (red[w] == bv && redi[w] < bx)) {
          bv = red[w];
          bx = redi[w];
        }
      if (!(bv > 0.0) || !isfinite(bv) || bx >= m) {
        s_bad = 1;
        bx = k;
      }
      s_piv = bx;
    }
    __syncthreads();
    const int pv = s_piv;
    if (pv != k)
      for (int c = k + threadIdx.x; c < ld; c += kMiBlock) {
        const double t = A[k * ld + c];
        A[k * ld + c] = A[pv * ld + c];
        A[pv * ld + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[k * ld + k];
    const int w = ld - k - 1;  // trailing columns k+1 .. ld-1
    const int rows = m - k - 1;
    for (int idx = threadIdx.x; idx < rows * w; idx += kMiBlock) {
      const int i = k + 1 + idx / w, c = k + 1 + idx % w;
      A[i * ld + c] = fma(-A[i * ld + k] * inv, A[k * ld + c], A[i * ld + c]);
    }
    __syncthreads();
  }
  // trailing upper triangle: x_{m-1}, then x_{m-2} for coupled items
  if (threadIdx.x == 0) {
    double x[2][2];
    bool bad = s_bad != 0;
    for (int b = 0; b < K; ++b) {
      const double u11 = A[(m - 1) * ld + (m - 1)];
      const double x1 = A[(m - 1) * ld + m + b] / u11;
      x[K - 1][b] = x1;
      if (K == 2) {
        const double u00 = A[(m - 2) * ld + (m - 2)], u01 = A[(m - 2) * ld + (m - 1)];
        x[0][b] = (A[(m - 2) * ld + m + b] - u01 * x1) / u00;
      }
    }
    // K_ab(p) = x[a][b]; symmetrised (K is symmetric, the solve is not exactly)
    double km[2][2];
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) km[a][b] = 0.5 * (x[a][b] + x[b][a]);
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) {
        if (!isfinite(km[a][b])) bad = true;
        kmat[it.k_off + (int64_t)e * K * K + a * K + b] = km[a][b];
      }
    // S = (1 - i h K)(1 + i h K)^-1, h = pi p / 2 (App. A; Sec. 2.1 K-matrix form)
    const double h = 0.5 * kPi * p;
    double d[2] = {0.0, 0.0}, eps = 0.0, ls = 0.0;
    if (K == 1) {
      // S = (1 - i h k)/(1 + i h k) = exp(-2 i atan(h k)), delta = -atan(h k)
      const double dd = -atan(h * km[0][0]);
      d[0] = dd;
      ls = 1.0 - cos(2.0 * dd);
    } else {
      // 2 x 2: M = 1 + i h K, S = (2 - M) M^-1 = 2 M^-1 - 1
      const double ar = 1.0, ai = h * km[0][0], br = 0.0, bi = h * km[0][1], dr = 1.0, di = h * km[1][1];
      // det = (1 + i h K00)(1 + i h K11) + h^2 K01^2
      const double detr = ar * dr - ai * di - (br * br - bi * bi);
      const double deti = ar * di + ai * dr - 2.0 * br * bi;
      const double dn = detr * detr + deti * deti;
      // M^-1 = [[d, -b], [-b, a]] / det
      auto cdiv = [&](double xr, double xi, double& yr, double& yi) {
        yr = (xr * detr + xi * deti) / dn;
        yi = (xi * detr - xr * deti) / dn;
      };
      double m00r, m00i, m01r, m01i, m11r, m11i;
      cdiv(dr, di, m00r, m00i);
      cdiv(-br, -bi, m01r, m01i);
      cdiv(ar, ai, m11r, m11i);
      const double s00r = 2.0 * m00r - 1.0, s00i = 2.0 * m00i;
      const double s11r = 2.0 * m11r - 1.0, s11i = 2.0 * m11i;
      const double s01r = 2.0 * m01r, s01i = 2.0 * m01i;
      d[0] = 0.5 * atan2(s00i, s00r);
      d[1] = 0.5 * atan2(s11i, s11r);
      const double ph = d[0] + d[1];
      double xx = s01i * cos(ph) - s01r * sin(ph);
      xx = xx > 1.0 ? 1.0 : (xx < -1.0 ? -1.0 : xx);
      eps = 0.5 * asin(xx);
      ls = (1.0 - s00r) + (1.0 - s11r);
    }
    for (int a = 0; a < K; ++a) delta[it.d_off + (int64_t)e * K + a] = bad ? NAN : d[a] * kRadToDeg;
    mix[it.m_off + e] = bad ? NAN : eps * kRadToDeg;
    loss[(int64_t)item * ne + e] = bad ? NAN : (2.0 * it.J + 1.0) * ls;
    if (bad) atomicMin(&status[item], (int)WPCD_ERR_NUMERIC);
  }
}

// sigma(p_e) = 10 pi/(2 p^2) sum over the sample's items of their terms [mb]
__global__ __launch_bounds__(256) void mi_sigma_kernel(const int32_t* __restrict__ sample_ptr,
                                                       const int32_t* __restrict__ sample_items,
                                                       const double* __restrict__ pts, int nq, int ne,
                                                       const double* __restrict__ loss, double* __restrict__ sigma) {
  const int s = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double p = pts[nq + e];
  double acc = 0.0;
  for (int q = sample_ptr[s]; q < sample_ptr[s + 1]; ++q) acc += loss[(int64_t)sample_items[q] * ne + e];
  sigma[(int64_t)s * ne + e] = 10.0 * kPi / (2.0 * p * p) * acc;
}

__global__ void mi_status_init_kernel(int32_t* status, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) status[i] = 0;
}

}  // namespace

size_t mi_lds_bytes(int nq, int K) {
  const int m = K * (nq + 1);
  return (size_t)m * (size_t)(m + K) * sizeof(double);
}

hipError_t launch_mi_solve(const MiItemDev* items, int n_items, int nq, int ne, int max_nch, const double* qw,
                           const double* pts, double cutoff, const double* u, double* kmat, double* delta,
                           double* mix, double* loss, const int32_t* sample_ptr, const int32_t* sample_items,
                           int n_samples, double* sigma, int32_t* status, hipStream_t s) {
  if (nq < 1 || nq > kMaxMiNq || ne < 1 || ne > 65535 || n_items > 65535) return hipErrorInvalidValue;
  const size_t lds = mi_lds_bytes(nq, max_nch);
  if (lds > 160 * 1024 - 4096) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mi_solve_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mi_status_init_kernel, dim3((n_items + 255) / 256), dim3(256), 0, s, status, n_items);
  hipLaunchKernelGGL(mi_solve_kernel, dim3(ne, n_items), dim3(kMiBlock), lds, s, items, nq, ne, qw, pts, cutoff, u,
                     kmat, delta, mix, loss, status);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_samples > 0 && sigma) {
    hipLaunchKernelGGL(mi_sigma_kernel, dim3((ne + 255) / 256, n_samples), dim3(256), 0, s, sample_ptr, sample_items,
                       pts, nq, ne, loss, sigma);
  }
  return hipGetLastError();
}

}  // namespace wpcd
