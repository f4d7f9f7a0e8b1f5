// S-matrix, phase shifts and total cross sections (App. A; Sec. 3.1 operator
// transfer; Sec. 5.1.1 mid-point interpolation).  All FP64.
#include "internal.h"

namespace wpcd {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRadToDeg = 57.295779513082320876798;
constexpr double kMnMeV = 938.918;
constexpr double kHbarcMeVfm = 197.327;

// One thread per (bin, item): t = T/(dk kbar^2), S = 1 - i pi kbar t,
// delta_a = arg(S_aa)/2, eps = asin(Im(Sbar12 exp(-i(d0+d1))))/2.
__global__ __launch_bounds__(256) void observables_kernel(const ItemDev* __restrict__ items, int item0,
                                                          const GridDev* __restrict__ grids,
                                                          const double* __restrict__ t, double* __restrict__ delta,
                                                          double* __restrict__ mix, double* __restrict__ s_dev) {
  const ItemDev it = items[item0 + blockIdx.y];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= it.N) return;
  const GridDev g = grids[it.grid];
  const int K = it.nch;
  const double fac = kPi / (g.dk[k] * g.kbar[k]);  // pi kbar / (dk kbar^2)
  const double* tk = t + it.t_off + 2 * (int64_t)k * K * K;
  double sre[2][2], sim[2][2];
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      const double tr = tk[2 * (a * K + b)], ti = tk[2 * (a * K + b) + 1];
      sre[a][b] = (a == b ? 1.0 : 0.0) + fac * ti;
      sim[a][b] = -fac * tr;
    }
  double d[2];
  for (int a = 0; a < K; ++a) {
    d[a] = 0.5 * atan2(sim[a][a], sre[a][a]);
    delta[it.d_off + (int64_t)k * K + a] = d[a] * kRadToDeg;
    if (s_dev) s_dev[it.d_off + (int64_t)k * K + a] = 1.0 - hypot(sre[a][a], sim[a][a]);
  }
  double e = 0.0;
  if (K == 2) {
    const double br = 0.5 * (sre[0][1] + sre[1][0]);
    const double bi = 0.5 * (sim[0][1] + sim[1][0]);
    const double ph = d[0] + d[1];
    double x = bi * cos(ph) - br * sin(ph);
    x = x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x);
    e = 0.5 * asin(x) * kRadToDeg;
  }
  mix[it.m_off + k] = e;
}

// One work-group per sample; threads over the T_lab list (at most
// 4*kSigBlock energies per sample).  Every item of the
// sample is unwrapped modulo 180 degrees from its lowest bin upwards (one
// thread per orbital channel), the mixing angle follows the parity of the
// shifts applied to its two phases, then each thread interpolates linearly in
// q between the bracketing midpoints and accumulates (2J+1) sum_a (1 - Re S_aa).
constexpr int kSigBlock = 256;
constexpr int kSigMaxBins = 1200;

__global__ __launch_bounds__(kSigBlock) void sigma_kernel(const ItemDev* __restrict__ items,
                                                          const int32_t* __restrict__ sample_ptr,
                                                          const int32_t* __restrict__ sample_items,
                                                          const GridDev* __restrict__ grids,
                                                          const double* __restrict__ delta,
                                                          const double* __restrict__ mix,
                                                          const double* __restrict__ tlab,
                                                          const int32_t* __restrict__ tlab_off, int n_tlab,
                                                          double* __restrict__ sigma) {
  __shared__ double dl[2][kSigMaxBins];
  __shared__ double mx[kSigMaxBins];
  __shared__ int sh[2][kSigMaxBins];
  const int smp = blockIdx.x;
  const int i0 = sample_ptr[smp], i1 = sample_ptr[smp + 1];
  // the sample's energies: its own slice of a packed list, or the shared list
  if (tlab_off) {
    const int j0 = tlab_off[smp];
    n_tlab = tlab_off[smp + 1] - j0;
    tlab += j0;
    sigma += j0;
  } else {
    sigma += (int64_t)smp * n_tlab;
  }
  // each thread owns T_lab indices j = tid, tid + kSigBlock, ...
  constexpr int kPer = 4;  // up to kPer*kSigBlock energies per sample
  double acc[kPer];
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
  for (int ii = i0; ii < i1; ++ii) {
    const ItemDev it = items[sample_items[ii]];
    const GridDev g = grids[it.grid];
    const int N = it.N, K = it.nch;
    __syncthreads();
    if (threadIdx.x < K) {
      const int a = threadIdx.x;
      const double* dp = delta + it.d_off;
      double prev = dp[a];
      dl[a][0] = prev;
      sh[a][0] = 0;
      for (int k = 1; k < N; ++k) {
        const double raw = dp[(int64_t)k * K + a];
        const double s = rint((prev - raw) / 180.0);
        prev = raw + 180.0 * s;
        dl[a][k] = prev;
        sh[a][k] = (int)s;
      }
    }
    __syncthreads();
    if (K == 2)
      for (int k = threadIdx.x; k < N; k += kSigBlock)
        mx[k] = (((sh[0][k] + sh[1][k]) & 1) ? -1.0 : 1.0) * mix[it.m_off + k];
    __syncthreads();
    const double* kb = g.kbar;
    const double kmax = g.kb[N];
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kSigBlock;
      if (j >= n_tlab) break;
      const double p = sqrt(kMnMeV * tlab[j] / 2.0) / kHbarcMeVfm;
      if (!(p > 0.0) || p > kmax) {
        acc[q] = NAN;
        continue;
      }
      // i = number of midpoints <= p, clamped to [1, N-1]
      int lo = 0, hi = N;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (kb[mid] <= p) lo = mid + 1;
        else hi = mid;
      }
      int i = lo < 1 ? 1 : (lo > N - 1 ? N - 1 : lo);
      const double x0 = kb[i - 1], x1 = kb[i];
      const double f = (p - x0) / (x1 - x0);
      double loss = 0.0;
      if (K == 1) {
        const double d = (dl[0][i - 1] + (dl[0][i] - dl[0][i - 1]) * f) / kRadToDeg;
        loss = 1.0 - cos(2.0 * d);
      } else {
        const double e = (mx[i - 1] + (mx[i] - mx[i - 1]) * f) / kRadToDeg;
        for (int a = 0; a < 2; ++a) {
          const double d = (dl[a][i - 1] + (dl[a][i] - dl[a][i - 1]) * f) / kRadToDeg;
          loss += 1.0 - cos(2.0 * e) * cos(2.0 * d);
        }
      }
      acc[q] += (2.0 * it.J + 1.0) * loss;
    }
  }
  for (int q = 0; q < kPer; ++q) {
    const int j = threadIdx.x + q * kSigBlock;
    if (j >= n_tlab) break;
    const double p = sqrt(kMnMeV * tlab[j] / 2.0) / kHbarcMeVfm;
    sigma[j] = 10.0 * kPi / (2.0 * p * p) * acc[q];
  }
}

}  // namespace

hipError_t launch_observables(const ItemDev* items, int n_items, int max_nbins, const GridDev* grids,
                              const double* t, double* delta, double* mix, double* s_dev, hipStream_t s) {
  const unsigned gx = (unsigned)((max_nbins + 255) / 256);
  for (int i0 = 0; i0 < n_items; i0 += 65535) {
    const unsigned gy = (unsigned)((n_items - i0) < 65535 ? (n_items - i0) : 65535);
    hipLaunchKernelGGL(observables_kernel, dim3(gx, gy), dim3(256), 0, s, items, i0, grids, t, delta, mix, s_dev);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_sigma(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                        int n_samples, const GridDev* grids, const double* delta, const double* mix,
                        const double* tlab, const int32_t* tlab_off, int n_tlab, double* sigma, hipStream_t s) {
  if (n_tlab > 4 * kSigBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sigma_kernel, dim3(n_samples), dim3(kSigBlock), 0, s, items, sample_ptr, sample_items, grids,
                     delta, mix, tlab, tlab_off, n_tlab, sigma);
  return hipGetLastError();
}

}  // namespace wpcd
