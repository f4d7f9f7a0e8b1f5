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

// The phases of one item unwrapped modulo 180 degrees from its lowest bin up
// (dl, one thread per orbital channel; sh the multiples of 180 applied) and
// its mixing angle with the sign of the parity of the two shifts (mx).  Called
// by the whole work-group; begins and ends with a barrier.
__device__ void unwrap_item(const ItemDev& it, const double* __restrict__ delta, const double* __restrict__ mix,
                            double (*dl)[kSigMaxBins], int (*sh)[kSigMaxBins], double* mx) {
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
    for (int k = threadIdx.x; k < N; k += blockDim.x)
      mx[k] = (((sh[0][k] + sh[1][k]) & 1) ? -1.0 : 1.0) * mix[it.m_off + k];
  __syncthreads();
}

// (2J+1) sum_a (1 - Re S_aa) at momentum p from the unwrapped phases, linear
// in q between the abscissae x (N of them, ascending; the end segments
// extrapolated), S rebuilt in the Stapp form.
template <class X>
__device__ double item_loss(const ItemDev& it, X x, double p, const double (*dl)[kSigMaxBins], const double* mx) {
  const int N = it.N, K = it.nch;
  // i = number of abscissae <= p, clamped to [1, N-1]
  int lo = 0, hi = N;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x(mid) <= p) lo = mid + 1;
    else hi = mid;
  }
  const int i = lo < 1 ? 1 : (lo > N - 1 ? N - 1 : lo);
  const double x0 = x(i - 1), x1 = x(i);
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
  return (2.0 * it.J + 1.0) * loss;
}

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
    unwrap_item(it, delta, mix, dl, sh, mx);
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
      acc[q] += item_loss(it, [kb](int m) { return kb[m]; }, p, dl, mx);
    }
  }
  for (int q = 0; q < kPer; ++q) {
    const int j = threadIdx.x + q * kSigBlock;
    if (j >= n_tlab) break;
    const double p = sqrt(kMnMeV * tlab[j] / 2.0) / kHbarcMeVfm;
    sigma[j] = 10.0 * kPi / (2.0 * p * p) * acc[q];
  }
}

// Interpolation-point bands (Sec. 5.1.1): the phases of bin i are placed at
// q_i = k_{i-1} + f (k_i - k_{i-1}) for every fraction f of the list, sigma is
// evaluated for each f as in sigma_kernel, and the lowest and highest values
// over f are written.  One work-group per sample, one thread per energy.
constexpr int kBandMaxFrac = 16;

__global__ __launch_bounds__(kSigBlock) void sigma_band_kernel(
    const ItemDev* __restrict__ items, const int32_t* __restrict__ sample_ptr, const int32_t* __restrict__ sample_items,
    const GridDev* __restrict__ grids, const double* __restrict__ delta, const double* __restrict__ mix,
    const double* __restrict__ tlab, int n_tlab, const double* __restrict__ fracs, int n_frac,
    double* __restrict__ sigma_lo, double* __restrict__ sigma_hi) {
  __shared__ double dl[2][kSigMaxBins];
  __shared__ double mx[kSigMaxBins];
  __shared__ int sh[2][kSigMaxBins];
  __shared__ double fr[kBandMaxFrac];
  const int smp = blockIdx.x;
  const int i0 = sample_ptr[smp], i1 = sample_ptr[smp + 1];
  if (threadIdx.x < n_frac) fr[threadIdx.x] = fracs[threadIdx.x];
  const int j = threadIdx.x;
  const double p = j < n_tlab ? sqrt(kMnMeV * tlab[j] / 2.0) / kHbarcMeVfm : 1.0;
  double acc[kBandMaxFrac];
#pragma unroll
  for (int f = 0; f < kBandMaxFrac; ++f) acc[f] = 0.0;
  bool out = !(p > 0.0);
  for (int ii = i0; ii < i1; ++ii) {
    const ItemDev it = items[sample_items[ii]];
    const GridDev g = grids[it.grid];
    unwrap_item(it, delta, mix, dl, sh, mx);
    if (j >= n_tlab) continue;
    const double* kb = g.kb;
    out = out || p > kb[it.N];
#pragma unroll
    for (int f = 0; f < kBandMaxFrac; ++f) {
      if (f >= n_frac) break;
      const double fv = fr[f];
      acc[f] += item_loss(it, [kb, fv](int m) { return kb[m] + fv * (kb[m + 1] - kb[m]); }, p, dl, mx);
    }
  }
  if (j >= n_tlab) return;
  double lo = acc[0], hi = acc[0];
#pragma unroll
  for (int f = 1; f < kBandMaxFrac; ++f) {
    if (f >= n_frac) break;
    lo = fmin(lo, acc[f]);
    hi = fmax(hi, acc[f]);
  }
  const double sc = 10.0 * kPi / (2.0 * p * p);
  sigma_lo[(int64_t)smp * n_tlab + j] = out ? NAN : sc * lo;
  sigma_hi[(int64_t)smp * n_tlab + j] = out ? NAN : sc * hi;
}

// ------------------------------------------------------- spin observables
// <l m1, 1 m2 | J m1 + m2> (spin-1 coupling, Condon-Shortley phase) and the
// spin-0 case <l m1, 0 0 | J m1> = delta_{lJ}.
__device__ double cg_spin(int l, int m1, int s, int m2, int J) {
  const int M = m1 + m2;
  if (m1 > l || -m1 > l || M > J || -M > J) return 0.0;
  if (s == 0) return (J == l && m2 == 0) ? 1.0 : 0.0;
  const double j = l, m = M;
  if (J == l + 1) {
    if (m2 == 1) return sqrt((j + m) * (j + m + 1) / ((2 * j + 1) * (2 * j + 2)));
    if (m2 == 0) return sqrt((j - m + 1) * (j + m + 1) / ((2 * j + 1) * (j + 1)));
    return sqrt((j - m) * (j - m + 1) / ((2 * j + 1) * (2 * j + 2)));
  }
  if (l == 0) return 0.0;
  if (J == l) {
    if (m2 == 1) return -sqrt((j + m) * (j - m + 1) / (2 * j * (j + 1)));
    if (m2 == 0) return m / sqrt(j * (j + 1));
    return sqrt((j - m) * (j + m + 1) / (2 * j * (j + 1)));
  }
  if (J == l - 1) {
    if (m2 == 1) return sqrt((j - m) * (j - m + 1) / (2 * j * (2 * j + 1)));
    if (m2 == 0) return -sqrt((j - m) * (j + m) / (j * (2 * j + 1)));
    return sqrt((j + m + 1) * (j + m) / (2 * j * (2 * j + 1)));
  }
  return 0.0;
}

// Y_l^m(theta, 0), |m| <= 2, Condon-Shortley phase: associated Legendre
// P_l^|m| by the upward recurrence from P_|m|^|m| = (2|m|-1)!! sin^|m|.
__device__ double ylm_theta(int l, int m, double ct, double st) {
  const int am = m < 0 ? -m : m;
  if (am > l) return 0.0;
  double pmm = 1.0;
  for (int k = 1; k <= am; ++k) pmm *= (2 * k - 1) * st;
  double plm = pmm;
  if (l > am) {
    double p0 = pmm, p1 = ct * (2 * am + 1) * pmm;
    for (int ll = am + 2; ll <= l; ++ll) {
      const double p2 = ((2 * ll - 1) * ct * p1 - (ll + am - 1) * p0) / (ll - am);
      p0 = p1;
      p1 = p2;
    }
    plm = p1;
  }
  // sqrt((2l+1)/(4 pi) (l-am)!/(l+am)!)
  double r = 1.0;
  for (int k = l - am + 1; k <= l + am; ++k) r *= k;
  const double y = ((am & 1) ? -1.0 : 1.0) * sqrt((2 * l + 1) / (4.0 * kPi) / r) * plm;
  return (m < 0 && (am & 1)) ? -y : y;
}

// Spin-scattering matrix, Saclay amplitudes and dsigma/dOmega (App. A) per
// sample, energy and angle.  One work-group per sample; thread tasks over
// (energy, angle).  Per item the phases are unwrapped and interpolated at p
// as in sigma_kernel, S rebuilt in the Stapp form, and each task adds the
// item's partial-wave terms
//   (2 pi/(i p)) sqrt((2l+1)/(4 pi)) Y_{l'}^{ms-ms'} <l' ms-ms', s ms'|J ms>
//   <l 0, s ms|J ms> (S_{l'l} - delta_{l'l})
// to the six independent M elements: M^0_00 and M^1_{11, 10, 1-1, 01, 00}.
// Then a = (M11 + M00 - M1-1)/2, b = (M11 + Ms + M1-1)/2,
// c = (M11 - Ms + M1-1)/2, d = -(M10 + M01)/(sqrt2 sin) or (M00 - a)/cos
// (the larger denominator), e = i (M01 - M10)/sqrt2, and
// dsigma/dOmega = (|a|^2 + ... + |e|^2)/2, in fm and 10 mb/sr.
constexpr int kSacPer = 4;  // tasks per thread: at most kSacPer * kSigBlock (energy, angle) pairs
__global__ __launch_bounds__(kSigBlock) void saclay_kernel(const ItemDev* __restrict__ items,
                                                           const int32_t* __restrict__ sample_ptr,
                                                           const int32_t* __restrict__ sample_items,
                                                           const GridDev* __restrict__ grids,
                                                           const double* __restrict__ delta,
                                                           const double* __restrict__ mix,
                                                           const double* __restrict__ tlab, int n_tlab,
                                                           const double* __restrict__ theta_deg, int n_theta,
                                                           double* __restrict__ amp, double* __restrict__ dsdo) {
  __shared__ double dl[2][kSigMaxBins];
  __shared__ double mx[kSigMaxBins];
  __shared__ int sh[2][kSigMaxBins];
  const int smp = blockIdx.x;
  const int i0 = sample_ptr[smp], i1 = sample_ptr[smp + 1];
  const int ntask = n_tlab * n_theta;
  // accumulators: M^0_00, M^1_11, M^1_10, M^1_1-1, M^1_01, M^1_00 (re, im)
  double acc[kSacPer][6][2];
  for (int q = 0; q < kSacPer; ++q)
    for (int k = 0; k < 6; ++k) acc[q][k][0] = acc[q][k][1] = 0.0;
  for (int ii = i0; ii < i1; ++ii) {
    const ItemDev it = items[sample_items[ii]];
    const GridDev g = grids[it.grid];
    const int N = it.N, K = it.nch;
    unwrap_item(it, delta, mix, dl, sh, mx);
    const double* kb = g.kbar;
    const double kmax = g.kb[N];
    const int s = it.spin, J = it.J;
    int ls[2];
    ls[0] = it.l0;
    ls[1] = it.l0 + 2;
    for (int q = 0; q < kSacPer; ++q) {
      const int task = threadIdx.x + q * kSigBlock;
      if (task >= ntask) break;
      const int ie = task / n_theta, jt = task - ie * n_theta;
      const double p = sqrt(kMnMeV * tlab[ie] / 2.0) / kHbarcMeVfm;
      if (!(p > 0.0) || p > kmax) {
        acc[q][0][0] = NAN;
        continue;
      }
      int lo = 0, hi = N;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (kb[mid] <= p) lo = mid + 1;
        else hi = mid;
      }
      const int i = lo < 1 ? 1 : (lo > N - 1 ? N - 1 : lo);
      const double f = (p - kb[i - 1]) / (kb[i] - kb[i - 1]);
      // S of the item at p (Stapp form; S[l' index][l index])
      double sre[2][2], sim[2][2];
      double d0 = (dl[0][i - 1] + (dl[0][i] - dl[0][i - 1]) * f) / kRadToDeg;
      if (K == 1) {
        sre[0][0] = cos(2.0 * d0);
        sim[0][0] = sin(2.0 * d0);
      } else {
        const double d1 = (dl[1][i - 1] + (dl[1][i] - dl[1][i - 1]) * f) / kRadToDeg;
        const double e = (mx[i - 1] + (mx[i] - mx[i - 1]) * f) / kRadToDeg;
        const double c2 = cos(2.0 * e), s2 = sin(2.0 * e);
        sre[0][0] = c2 * cos(2.0 * d0);
        sim[0][0] = c2 * sin(2.0 * d0);
        sre[1][1] = c2 * cos(2.0 * d1);
        sim[1][1] = c2 * sin(2.0 * d1);
        // i sin(2e) exp(i (d0 + d1))
        sre[0][1] = sre[1][0] = -s2 * sin(d0 + d1);
        sim[0][1] = sim[1][0] = s2 * cos(d0 + d1);
      }
      const double th = theta_deg[jt] / kRadToDeg;
      const double ct = cos(th), st = sin(th);
      // (2 pi/(i p)) z = (2 pi/p)(Im z, -Re z)
      const double pref = 2.0 * kPi / p;
      // the six elements: (s, ms, ms')
      const int es[6] = {0, 1, 1, 1, 1, 1}, ems[6] = {0, 1, 1, 1, 0, 0}, emp[6] = {0, 1, 0, -1, 1, 0};
      for (int k = 0; k < 6; ++k) {
        if (es[k] != s) continue;
        const int ms = ems[k], msp = emp[k];
        double zr = 0.0, zi = 0.0;
        for (int ia = 0; ia < K; ++ia) {
          const int l = ls[ia];
          const double cin = cg_spin(l, 0, s, ms, J);
          if (cin == 0.0) continue;
          for (int ib = 0; ib < K; ++ib) {
            const int lp = ls[ib];
            const double cout = cg_spin(lp, ms - msp, s, msp, J);
            if (cout == 0.0) continue;
            const double w = sqrt((2 * l + 1) / (4.0 * kPi)) * cin * cout * ylm_theta(lp, ms - msp, ct, st);
            zr += w * (sre[ib][ia] - (ia == ib ? 1.0 : 0.0));
            zi += w * sim[ib][ia];
          }
        }
        acc[q][k][0] += pref * zi;
        acc[q][k][1] -= pref * zr;
      }
    }
  }
  for (int q = 0; q < kSacPer; ++q) {
    const int task = threadIdx.x + q * kSigBlock;
    if (task >= ntask) break;
    const int jt = task % n_theta;
    const double th = theta_deg[jt] / kRadToDeg;
    const double ct = cos(th), st = sin(th);
    double (*M)[2] = acc[q];
    // amplitudes (re, im): a, b, c, d, e
    double am[5][2];
    for (int c = 0; c < 2; ++c) {
      am[0][c] = 0.5 * (M[1][c] + M[5][c] - M[3][c]);
      am[1][c] = 0.5 * (M[1][c] + M[0][c] + M[3][c]);
      am[2][c] = 0.5 * (M[1][c] - M[0][c] + M[3][c]);
      am[3][c] = fabs(st) >= fabs(ct) ? -(M[2][c] + M[4][c]) / (sqrt(2.0) * st) : (M[5][c] - am[0][c]) / ct;
    }
    // e = i (M01 - M10)/sqrt2
    am[4][0] = -(M[4][1] - M[2][1]) / sqrt(2.0);
    am[4][1] = (M[4][0] - M[2][0]) / sqrt(2.0);
    double ds = 0.0;
    for (int k = 0; k < 5; ++k) ds += am[k][0] * am[k][0] + am[k][1] * am[k][1];
    const int64_t o = (int64_t)smp * ntask + task;
    dsdo[o] = 10.0 * 0.5 * ds;
    if (amp)
      for (int k = 0; k < 5; ++k) {
        amp[10 * o + 2 * k] = am[k][0];
        amp[10 * o + 2 * k + 1] = am[k][1];
      }
  }
}

}  // namespace

hipError_t launch_saclay(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                         int n_samples, const GridDev* grids, const double* delta, const double* mix,
                         const double* tlab, int n_tlab, const double* theta_deg, int n_theta, double* amp,
                         double* dsdo, hipStream_t s) {
  if ((int64_t)n_tlab * n_theta > (int64_t)kSacPer * kSigBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(saclay_kernel, dim3(n_samples), dim3(kSigBlock), 0, s, items, sample_ptr, sample_items, grids,
                     delta, mix, tlab, n_tlab, theta_deg, n_theta, amp, dsdo);
  return hipGetLastError();
}

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

hipError_t launch_sigma_band(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                             int n_samples, const GridDev* grids, const double* delta, const double* mix,
                             const double* tlab, int n_tlab, const double* fracs, int n_frac, double* sigma_lo,
                             double* sigma_hi, hipStream_t s) {
  if (n_tlab < 1 || n_tlab > kSigBlock || n_frac < 1 || n_frac > kBandMaxFrac) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sigma_band_kernel, dim3(n_samples), dim3(kSigBlock), 0, s, items, sample_ptr, sample_items,
                     grids, delta, mix, tlab, n_tlab, fracs, n_frac, sigma_lo, sigma_hi);
  return hipGetLastError();
}

}  // namespace wpcd
