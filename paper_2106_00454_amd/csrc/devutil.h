// Device helpers shared by the eigensolver kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wpcd {

// ---------------------------------------------------------------------------
// Sums over aligned groups of G lanes (G = 2 ... 64) with DPP lane swizzles.
// Every lane of a group ends with the bitwise-same total: each butterfly stage
// adds the same two partial sums in either order, and IEEE addition is
// commutative, so control decisions taken on the result are group-uniform.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kQuadXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// Groups of 32 and 64 lanes add the other 16-lane rows with xor shuffles
// (each pair of lanes again adds the same two values).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
  if (G >= 2) v += dpp_f32<kQuadXor1>(v);
  if (G >= 4) v += dpp_f32<kQuadXor2>(v);
  if (G >= 8) v += dpp_f32<kRowHalfMirror>(v);
  if (G >= 16) v += dpp_f32<kRowMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
  if (G >= 2) v += dpp_f64<kQuadXor1>(v);
  if (G >= 4) v += dpp_f64<kQuadXor2>(v);
  if (G >= 8) v += dpp_f64<kRowHalfMirror>(v);
  if (G >= 16) v += dpp_f64<kRowMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Sum over the 64 lanes of a wavefront, in every lane (a scalar): row sums
// by the DPP butterfly above, then row_bcast:15 adds row 0 to row 1 and row
// 2 to row 3 (rows 1 and 3 written), row_bcast:31 adds rows 0-1 to rows 2-3
// (rows 2 and 3 written), and lane 63 holds the total, read as a scalar.  No
// LDS traffic (a __shfl_xor butterfly takes six ds_bpermute round trips).
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows_f64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffLL), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float wave_total(float v) {
  v = group_sum<16>(v);
  v += dpp_rows_f32<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_rows_f32<0x143, 0xC>(v);  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double wave_total(double v) {
  v = group_sum<16>(v);
  v += dpp_rows_f64<0x142, 0xA>(v);
  v += dpp_rows_f64<0x143, 0xC>(v);
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Round-robin ("circle") ordering of a parallel Jacobi sweep over ne (even)
// indices: position 0 keeps index 0, position q >= 1 holds
// 1 + ((q - 1 + step) mod (ne - 1)); pairs are positions (i, ne-1-i).  Over
// ne-1 steps every unordered pair meets exactly once and the pairs of one step
// are disjoint, so they can be rotated concurrently (Sec. 4.2, parallel
// cyclic-order Jacobi; Golub & Van Loan, parallel ordering).
__device__ __forceinline__ int rr_index(int pos, int step, int ne) {
  if (pos == 0) return 0;
  int v = pos - 1 + step;
  const int m = ne - 1;
  v -= (v / m) * m;
  return 1 + v;
}

// Rotation of the one-sided (Hestenes) Jacobi method: with Gram entries
// al = |w_p|^2, be = |w_q|^2, ga = w_p.w_q, the plane rotation
//   w_p <- c w_p - s w_q,  w_q <- s w_p + c w_q
// with t = s/c the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (be-al)/(2ga),
// makes the two columns orthogonal.
template <typename T>
__device__ __forceinline__ void hestenes_rotation(T al, T be, T ga, T& c, T& s) {
  const T zeta = (be - al) / (T(2) * ga);
  const T t = copysign(T(1), zeta) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
  c = T(1) / sqrt(T(1) + t * t);
  s = c * t;
}

// One-sided cyclic Jacobi on the n columns of W (column-major, leading
// dimension ld) resident in LDS, executed by a whole work-group of BLOCK
// threads in lane groups of G; each group owns one column pair per step and
// keeps it in registers (RMAX >= ceil(n/G) rows per lane).  A pair is rotated
// while |w_p.w_q| > tol |w_p||w_q|.  rot_flag must point to max_sweeps zeroed
// shared ints; each records the largest rotated |w_p.w_q|/(|w_p||w_q|) of its
// sweep (as the bits of a non-negative float, so integer max is float max).
// The iteration ends after a sweep that rotated nothing or only pairs below
// 8 tol (rounding-level rotations that would otherwise recur).  Returns the
// number of sweeps run, or max_sweeps + 1 if the last allowed sweep still
// rotated larger pairs (not converged).  Ends with a barrier.
template <typename T, int BLOCK, int G, int RMAX>
__device__ int onesided_jacobi_lds(T* W, int n, int ld, T tol, T stop, int max_sweeps, int* rot_flag) {
  const int npair = (n + 1) >> 1;
  const int ne = npair << 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    for (int step = 0; step < ne - 1; ++step) {
      for (int pr = grp; pr < npair; pr += ngrp) {
        const int p = rr_index(pr, step, ne);
        const int q = rr_index(ne - 1 - pr, step, ne);
        if (p >= n || q >= n) continue;  // the padding index of odd n
        T* wp = W + (int64_t)p * ld;
        T* wq = W + (int64_t)q * ld;
        T xp[RMAX], xq[RMAX];
        T al = T(0), be = T(0), ga = T(0);
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
          const int r = lane + k * G;
          T a = T(0), b = T(0);
          if (r < n) {
            a = wp[r];
            b = wq[r];
          }
          xp[k] = a;
          xq[k] = b;
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
#pragma unroll
          for (int k = 0; k < RMAX; ++k) {
            const int r = lane + k * G;
            if (r < n) {
              wp[r] = c * xp[k] - s * xq[k];
              wq[r] = s * xp[k] + c * xq[k];
            }
          }
          if (lane == 0) atomicMax(&rot_flag[sweep], __float_as_int((float)(fabs(ga) / nab)));
        }
      }
      __syncthreads();
    }
    if (__int_as_float(rot_flag[sweep]) < (float)stop) return sweep + 1;
  }
  return max_sweeps + 1;
}

// rr_index for 0 <= pos < ne and 0 <= step < ne - 1, without a division.
__device__ __forceinline__ int rr_index_nodiv(int pos, int step, int ne) {
  if (pos == 0) return 0;
  int v = pos - 1 + step;
  if (v >= ne - 1) v -= ne - 1;
  return 1 + v;
}

// The same iteration with tracked column norms: nrm2 (n shared floats) holds
// |w_c|^2, recomputed exactly at the start of every sweep and updated after a
// rotation by the exact identities |w_p'|^2 = |w_p|^2 - t w_p.w_q and
// |w_q'|^2 = |w_q|^2 + t w_p.w_q (t = s/c), so a pair step computes one dot
// product instead of three.  FP32 only; the caller guarantees ld >= RMAX*G
// and zero rows n .. RMAX*G-1 in every column, so no row is guarded (the zero
// rows stay zero under rotations).  The rotation is formed with the hardware
// reciprocal and square-root instructions (about 1 ulp): only the angle
// depends on them; c and s are normalised by construction to 1 ulp, as with
// correctly rounded operations.  Same tolerance, stopping rule and return
// value as onesided_jacobi_lds; nrot (lane 0 of each group) counts the
// rotations the group applied.
template <int BLOCK, int G, int RMAX>
__device__ int onesided_jacobi_lds_tracked(float* W, int n, int ld, float tol, float stop, int max_sweeps, int* rot_flag,
                                           float* nrm2, int& nrot) {
  const int npair = (n + 1) >> 1;
  const int ne = npair << 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int c = grp; c < n; c += ngrp) {
      const float* col = W + c * ld + lane;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) s2 = fmaf(col[k * G], col[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm2[c] = s2;
    }
    __syncthreads();
    for (int step = 0; step < ne - 1; ++step) {
      for (int pr = grp; pr < npair; pr += ngrp) {
        const int p = rr_index_nodiv(pr, step, ne);
        const int q = rr_index_nodiv(ne - 1 - pr, step, ne);
        if (p >= n || q >= n) continue;  // the padding index of odd n
        float* wp = W + p * ld + lane;
        float* wq = W + q * ld + lane;
        float xp[RMAX], xq[RMAX];
        float ga = 0.f;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
          xp[k] = wp[k * G];
          xq[k] = wq[k * G];
          ga = fmaf(xp[k], xq[k], ga);
        }
        ga = group_sum<G>(ga);
        const float al = nrm2[p], be = nrm2[q];
        const float nab = __builtin_amdgcn_sqrtf(al * be);
        if (fabsf(ga) > tol * nab) {
          const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.f * ga);
          const float t = copysignf(1.f, zeta) *
                          __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(fmaf(zeta, zeta, 1.f)));
          const float c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
          const float s = c * t;
#pragma unroll
          for (int k = 0; k < RMAX; ++k) {
            wp[k * G] = c * xp[k] - s * xq[k];
            wq[k * G] = s * xp[k] + c * xq[k];
          }
          if (lane == 0) {
            nrm2[p] = al - t * ga;
            nrm2[q] = be + t * ga;
            atomicMax(&rot_flag[sweep], __float_as_int(fabsf(ga) * __builtin_amdgcn_rcpf(nab)));
            ++nrot;
          }
        }
      }
      __syncthreads();
    }
    if (__int_as_float(rot_flag[sweep]) < stop) return sweep + 1;
  }
  return max_sweeps + 1;
}

// Column-blocked iteration with tracked norms (FP32, LDS-resident W): the
// ordering of onesided_jacobi_blocked (pairs inside each block of B columns,
// then a round robin over blocks whose block-pair steps rotate the B*B cross
// pairs in B stages), the rotation arithmetic of onesided_jacobi_lds_tracked.
// A lane group holds its 2B columns and their squared norms in registers for
// the whole block step, so one barrier and one LDS round trip serve B*B
// rotations.  Rows: lane + k*G for k < RMAX; only the last k is guarded
// (rows >= n are skipped).  nrm2 holds the squared norms between steps.
template <int G, int RMAX, int NP, class IA, class IB, int B>
__device__ __forceinline__ void rotate_tracked(float (&xs)[B][RMAX], float (&ys)[B][RMAX], float (&ns)[B],
                                               float (&ms)[B], bool (&dx)[B], bool (&dy)[B], IA ia, IB ib,
                                               float tol, float& rmax, int& nrot) {
  float ga[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) ga[i] = 0.f;
#pragma unroll
  for (int k = 0; k < RMAX; ++k)
#pragma unroll
    for (int i = 0; i < NP; ++i) ga[i] = fmaf(xs[ia(i)][k], ys[ib(i)][k], ga[i]);
#pragma unroll
  for (int i = 0; i < NP; ++i) ga[i] = group_sum<G>(ga[i]);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const float al = ns[ia(i)], be = ms[ib(i)];
    const float nab = __builtin_amdgcn_sqrtf(al * be);
    if (fabsf(ga[i]) > tol * nab) {
      const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.f * ga[i]);
      const float t = copysignf(1.f, zeta) *
                      __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(fmaf(zeta, zeta, 1.f)));
      const float c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
      const float s = c * t;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) {
        const float a = xs[ia(i)][k], b = ys[ib(i)][k];
        xs[ia(i)][k] = c * a - s * b;
        ys[ib(i)][k] = s * a + c * b;
      }
      ns[ia(i)] = al - t * ga[i];
      ms[ib(i)] = be + t * ga[i];
      const float rel = fabsf(ga[i]) * __builtin_amdgcn_rcpf(nab);
      rmax = rel > rmax ? rel : rmax;
      dx[ia(i)] = true;
      dy[ib(i)] = true;
      if (threadIdx.x % G == 0) ++nrot;
    }
  }
}

template <int G, int RMAX, int B>
__device__ __forceinline__ void load_block(const float* W, float* nrm2, int blk, int n, int ld, int lane,
                                           float (&x)[B][RMAX], float (&nx)[B]) {
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int c = blk * B + i;
    const bool live = c < n;
    const float* col = W + (live ? c : 0) * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
      const bool ok = live && (k < RMAX - 1 || lane + k * G < n);
      x[i][k] = ok ? col[k * G] : 0.f;
    }
    nx[i] = live ? nrm2[c] : 0.f;
  }
}

template <int G, int RMAX, int B>
__device__ __forceinline__ void store_block(float* W, float* nrm2, int blk, int n, int ld, int lane,
                                            const float (&x)[B][RMAX], const float (&nx)[B], const bool (&d)[B]) {
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int c = blk * B + i;
    if (c >= n || !d[i]) continue;
    float* col = W + c * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane + k * G < n) col[k * G] = x[i][k];
    if (lane == 0) nrm2[c] = nx[i];
  }
}

template <int BLOCK, int G, int RMAX, int B>
__device__ int onesided_jacobi_blocked_tracked(float* W, int n, int ld, float tol, float stop, int max_sweeps,
                                               int* rot_flag,
                                               float* nrm2, int& nrot) {
  static_assert(B == 2 || B == 4, "block width");
  const int nb = (n + B - 1) / B;
  const int nbp = (nb + 1) >> 1;
  const int nbe = nbp << 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    float rmax = 0.f;
    // exact squared norms at the start of the sweep
    for (int c = grp; c < n; c += ngrp) {
      const float* col = W + c * ld + lane;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < RMAX - 1 || lane + k * G < n) s2 = fmaf(col[k * G], col[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm2[c] = s2;
    }
    __syncthreads();
    // pairs inside each block
    for (int blk = grp; blk < nb; blk += ngrp) {
      float x[B][RMAX], nx[B];
      bool dx[B];
      load_block<G, RMAX, B>(W, nrm2, blk, n, ld, lane, x, nx);
#pragma unroll
      for (int i = 0; i < B; ++i) dx[i] = false;
#pragma unroll
      for (int st = 0; st < B - 1; ++st) {
        auto col = [st](int q) { return q == 0 ? 0 : 1 + (q - 1 + st) % (B - 1); };
        rotate_tracked<G, RMAX, B / 2>(x, x, nx, nx, dx, dx, [&](int i) { return col(i); },
                                       [&](int i) { return col(B - 1 - i); }, tol, rmax, nrot);
      }
      store_block<G, RMAX, B>(W, nrm2, blk, n, ld, lane, x, nx, dx);
    }
    __syncthreads();
    for (int step = 0; step < nbe - 1; ++step) {
      for (int pr = grp; pr < nbp; pr += ngrp) {
        const int P = rr_index_nodiv(pr, step, nbe);
        const int Q = rr_index_nodiv(nbe - 1 - pr, step, nbe);
        if (P >= nb || Q >= nb) continue;  // the padding block of odd nb
        float x[B][RMAX], y[B][RMAX], nx[B], ny[B];
        bool dx[B], dy[B];
        load_block<G, RMAX, B>(W, nrm2, P, n, ld, lane, x, nx);
        load_block<G, RMAX, B>(W, nrm2, Q, n, ld, lane, y, ny);
#pragma unroll
        for (int i = 0; i < B; ++i) {
          dx[i] = false;
          dy[i] = false;
        }
#pragma unroll
        for (int st = 0; st < B; ++st)
          rotate_tracked<G, RMAX, B>(x, y, nx, ny, dx, dy, [](int i) { return i; },
                                     [st](int i) { return (i + st) % B; }, tol, rmax, nrot);
        store_block<G, RMAX, B>(W, nrm2, P, n, ld, lane, x, nx, dx);
        store_block<G, RMAX, B>(W, nrm2, Q, n, ld, lane, y, ny, dy);
      }
      __syncthreads();
    }
    if (lane == 0 && rmax > 0.f) atomicMax(&rot_flag[sweep], __float_as_int(rmax));
    __syncthreads();
    if (__int_as_float(rot_flag[sweep]) < stop) return sweep + 1;
  }
  return max_sweeps + 1;
}

// Scaled rotations for the blocked iteration: column j is stored as w~_j with
// w_j = d_j w~_j.  The rotation w_p' = c (w_p - t w_q), w_q' = c (w_q + t w_p)
// is applied as two in-place shears, w~_q <- w~_q + (t d_p/d_q) w~_p, then
// w~_p <- w~_p - (t c^2 d_q/d_p) w~_q (with the updated w~_q), and the scales
// d_p <- d_p / c, d_q <- c d_q: one FMA per element and column, no copies.
// Squared norms are tracked for the true columns w; the pair's inner product
// is d_p d_q (w~_p . w~_q).  The angle uses t = 2 g sgn(D) / (|D| +
// sqrt(D^2 + 4 g^2)), D = |w_q|^2 - |w_p|^2, g = w_p . w_q (the smaller of the
// two Jacobi angles), c = 1/sqrt(1 + t^2).  A scale outside [2^-12, 2^12] is
// folded back into its column (w~ *= d, d = 1), so the FP32 products stay far
// from overflow and underflow.
template <int G, int RMAX, int NP, class IA, class IB, int B>
__device__ __forceinline__ void rotate_scaled(float (&xs)[B][RMAX], float (&ys)[B][RMAX], float (&ns)[B],
                                              float (&ms)[B], float (&ds)[B], float (&es)[B], bool (&dx)[B],
                                              bool (&dy)[B], IA ia, IB ib, float tol2, float stop2, bool& big,
                                              int& nrot) {
  float ga[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) ga[i] = 0.f;
#pragma unroll
  for (int k = 0; k < RMAX; ++k)
#pragma unroll
    for (int i = 0; i < NP; ++i) ga[i] = fmaf(xs[ia(i)][k], ys[ib(i)][k], ga[i]);
#pragma unroll
  for (int i = 0; i < NP; ++i) ga[i] = group_sum<G>(ga[i]);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const float dp = ds[ia(i)], dq = es[ib(i)];
    const float pq = dp * dq;
    const float g = ga[i] * pq;
    const float al = ns[ia(i)], be = ms[ib(i)];
    const float ab = al * be, g2 = g * g;
    if (g2 > tol2 * ab) {
      const float D = be - al;
      const float t = copysignf(1.f, D) * (2.f * g) *
                      __builtin_amdgcn_rcpf(fabsf(D) + __builtin_amdgcn_sqrtf(fmaf(D, D, 4.f * g2)));
      const float u = fmaf(t, t, 1.f);
      const float c = __builtin_amdgcn_rsqf(u);
      const float r = t * __builtin_amdgcn_rcpf(pq);
      const float bq = r * dp * dp, ap = r * dq * dq * c * c;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) {
        ys[ib(i)][k] = fmaf(bq, xs[ia(i)][k], ys[ib(i)][k]);
        xs[ia(i)][k] = fmaf(-ap, ys[ib(i)][k], xs[ia(i)][k]);
      }
      ds[ia(i)] = dp * u * c;
      es[ib(i)] = c * dq;
      ns[ia(i)] = al - t * g;
      ms[ib(i)] = be + t * g;
      big = big || g2 > stop2 * ab;  // a rotation at or above the stopping threshold
      dx[ia(i)] = true;
      dy[ib(i)] = true;
      if (threadIdx.x % G == 0) ++nrot;
    }
  }
}

// Columns blk*B .. blk*B+B-1 (column n, the zero column of odd n, included);
// rows below (RMAX-1)*G are read unguarded (zero-padded up to there), the
// last row chunk is read in full (W has G spare floats at its end) and masked.
template <int G, int RMAX, int B>
__device__ __forceinline__ void load_block_scaled(const float* W, const float* nrm2, const float* dsc, int blk,
                                                  int n, int ld, int lane, float (&x)[B][RMAX], float (&nx)[B],
                                                  float (&d)[B]) {
  const bool last_ok = lane + (RMAX - 1) * G < n;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int c = blk * B + i;
    const float* col = W + c * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX - 1; ++k) x[i][k] = col[k * G];
    const float v = col[(RMAX - 1) * G];
    x[i][RMAX - 1] = last_ok ? v : 0.f;
    nx[i] = nrm2[c];
    d[i] = dsc[c];
  }
}

template <int G, int RMAX, int B>
__device__ __forceinline__ void store_block_scaled(float* W, float* nrm2, float* dsc, int blk, int n, int ld,
                                                   int lane, float (&x)[B][RMAX], const float (&nx)[B],
                                                   float (&d)[B], const bool (&dirty)[B]) {
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int c = blk * B + i;
    if (c >= n || !dirty[i]) continue;
    if (d[i] < 0x1p-12f || d[i] > 0x1p12f) {  // fold the scale back into the column
#pragma unroll
      for (int k = 0; k < RMAX; ++k) x[i][k] *= d[i];
      d[i] = 1.f;
    }
    float* col = W + c * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane + k * G < n) col[k * G] = x[i][k];
    if (lane == 0) {
      nrm2[c] = nx[i];
      dsc[c] = d[i];
    }
  }
}

// The blocked iteration of onesided_jacobi_blocked_tracked with scaled
// rotations (same ordering, skip test and stopping rule; rot_flag[sweep]
// becomes 1 when a rotation of the sweep reached the stopping threshold).  W holds nb*B
// columns (for odd n column n is zero and never rotates) and G spare floats
// after the last one.  On return the scales are folded into W, so its columns
// are the true w_j.
template <int BLOCK, int G, int RMAX, int B>
__device__ int onesided_jacobi_blocked_scaled(float* W, int n, int ld, float tol, float stop, int max_sweeps,
                                              int* rot_flag,
                                              float* nrm2, float* dsc, int& nrot) {
  static_assert(B == 2 || B == 4, "block width");
  const int nb = (n + B - 1) / B;
  const int nbp = (nb + 1) >> 1;
  const int nbe = nbp << 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  const float tol2 = tol * tol, stop2 = stop * stop;
  for (int c = threadIdx.x; c < nb * B; c += BLOCK) {
    dsc[c] = 1.f;
    nrm2[c] = 0.f;  // stays 0 for the zero column of odd n
  }
  int sweeps = max_sweeps + 1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    bool big = false;
    __syncthreads();
    // exact squared norms of the true columns at the start of the sweep
    for (int c = grp; c < n; c += ngrp) {
      const float* col = W + c * ld + lane;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < RMAX - 1 || lane + k * G < n) s2 = fmaf(col[k * G], col[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm2[c] = s2 * dsc[c] * dsc[c];
    }
    __syncthreads();
    for (int blk = grp; blk < nb; blk += ngrp) {
      float x[B][RMAX], nx[B], d[B];
      bool dx[B];
      load_block_scaled<G, RMAX, B>(W, nrm2, dsc, blk, n, ld, lane, x, nx, d);
#pragma unroll
      for (int i = 0; i < B; ++i) dx[i] = false;
#pragma unroll
      for (int st = 0; st < B - 1; ++st) {
        auto col = [st](int q) { return q == 0 ? 0 : 1 + (q - 1 + st) % (B - 1); };
        rotate_scaled<G, RMAX, B / 2>(x, x, nx, nx, d, d, dx, dx, [&](int i) { return col(i); },
                                      [&](int i) { return col(B - 1 - i); }, tol2, stop2, big, nrot);
      }
      store_block_scaled<G, RMAX, B>(W, nrm2, dsc, blk, n, ld, lane, x, nx, d, dx);
    }
    __syncthreads();
    for (int step = 0; step < nbe - 1; ++step) {
      for (int pr = grp; pr < nbp; pr += ngrp) {
        const int P = rr_index_nodiv(pr, step, nbe);
        const int Q = rr_index_nodiv(nbe - 1 - pr, step, nbe);
        if (P >= nb || Q >= nb) continue;  // the padding block of odd nb
        float x[B][RMAX], y[B][RMAX], nx[B], ny[B], dxs[B], dys[B];
        bool dx[B], dy[B];
        load_block_scaled<G, RMAX, B>(W, nrm2, dsc, P, n, ld, lane, x, nx, dxs);
        load_block_scaled<G, RMAX, B>(W, nrm2, dsc, Q, n, ld, lane, y, ny, dys);
#pragma unroll
        for (int i = 0; i < B; ++i) {
          dx[i] = false;
          dy[i] = false;
        }
#pragma unroll
        for (int st = 0; st < B; ++st)
          rotate_scaled<G, RMAX, B>(x, y, nx, ny, dxs, dys, dx, dy, [](int i) { return i; },
                                    [st](int i) { return (i + st) % B; }, tol2, stop2, big, nrot);
        store_block_scaled<G, RMAX, B>(W, nrm2, dsc, P, n, ld, lane, x, nx, dxs, dx);
        store_block_scaled<G, RMAX, B>(W, nrm2, dsc, Q, n, ld, lane, y, ny, dys, dy);
      }
      __syncthreads();
    }
    if (lane == 0 && big) rot_flag[sweep] = __float_as_int(1.f);  // any group may set it
    __syncthreads();
    if (__int_as_float(rot_flag[sweep]) < stop) {
      sweeps = sweep + 1;
      break;
    }
  }
  // fold the remaining scales into the columns
  __syncthreads();
  for (int c = grp; c < n; c += ngrp) {
    const float dc = dsc[c];
    if (dc == 1.f) continue;
    float* col = W + c * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane + k * G < n) col[k * G] *= dc;
  }
  __syncthreads();
  return sweeps;
}

// The iteration of onesided_jacobi_blocked_scaled (blocks of 2 columns,
// scaled rotations, tracked norms; same skip test, stopping rule and return
// value) in an ordering that lets every lane group keep one block in
// registers: a sweep splits the blocks [0, nb) into A = [0, h) and
// B = [h, nb), h = floor(nb / 2); for ceil(nb / 2) steps group g pairs A[g]
// with B[(g + s) mod |B|], so A[g] stays in its registers and only the B
// blocks pass through LDS; then A and B are split the same way, side by side
// (the left child keeps the first floor(|A| / 2) groups of its parent, the
// right child the next floor(|B| / 2)), down to blocks of one.  Every block
// pair meets once per sweep and the pairs of a step are disjoint; a sweep
// has sum_l ceil(ceil(nb / 2^l) / 2) steps (102 for nb = 100, against 99
// for the round-robin ordering) but moves one block per group and step
// through LDS instead of two.  At the start of every level the kept blocks
// go back to LDS before any group loads its next one (one barrier).
template <int BLOCK, int G, int RMAX>
__device__ int onesided_jacobi_keep_scaled(float* W, int n, int ld, float tol, float stop, int max_sweeps,
                                           int* rot_flag, float* nrm2, float* dsc, int& nrot) {
  constexpr int B = 2;
  const int nb = (n + B - 1) / B;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  static_assert(G * RMAX / (2 * B) <= ngrp, "every block pair of a step has a lane group");
  const float tol2 = tol * tol, stop2 = stop * stop;
  for (int c = threadIdx.x; c < nb * B; c += BLOCK) {
    dsc[c] = 1.f;
    nrm2[c] = 0.f;  // stays 0 for the zero column of odd n
  }
  int sweeps = max_sweeps + 1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    bool big = false;
    __syncthreads();
    // exact squared norms of the true columns at the start of the sweep
    for (int c = grp; c < n; c += ngrp) {
      const float* col = W + c * ld + lane;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < RMAX - 1 || lane + k * G < n) s2 = fmaf(col[k * G], col[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm2[c] = s2 * dsc[c] * dsc[c];
    }
    __syncthreads();
    // the pair inside each block
    for (int blk = grp; blk < nb; blk += ngrp) {
      float x[B][RMAX], nx[B], d[B];
      bool dx[B];
      load_block_scaled<G, RMAX, B>(W, nrm2, dsc, blk, n, ld, lane, x, nx, d);
#pragma unroll
      for (int i = 0; i < B; ++i) dx[i] = false;
      rotate_scaled<G, RMAX, 1>(x, x, nx, nx, d, d, dx, dx, [](int) { return 0; }, [](int) { return 1; }, tol2,
                                stop2, big, nrot);
      store_block_scaled<G, RMAX, B>(W, nrm2, dsc, blk, n, ld, lane, x, nx, d, dx);
    }
    // levels of the halving ordering
    float x[B][RMAX], nx[B], dxs[B];
    bool dx[B];
    int keep = -1;
    for (int lvl = 0, lmax = nb; lmax >= 2; ++lvl, lmax = (lmax + 1) >> 1) {
      // back to LDS with the kept block (every group), then this level's node
      if (keep >= 0) store_block_scaled<G, RMAX, B>(W, nrm2, dsc, keep, n, ld, lane, x, nx, dxs, dx);
      keep = -1;
      __syncthreads();
      int lo = 0, hi = nb, g0 = 0;
      bool mine = true;
      for (int l = 0; l < lvl; ++l) {
        const int len = hi - lo, h = len >> 1;
        if (grp < g0 + (h >> 1)) {
          hi = lo + h;
        } else if (grp < g0 + (h >> 1) + ((len - h) >> 1)) {
          g0 += h >> 1;
          lo += h;
        } else {
          mine = false;
          break;
        }
      }
      const int len = hi - lo, h = len >> 1, nbk = len - h, gl = grp - g0;
      mine = mine && len >= 2 && gl < h;
      if (mine) {
        keep = lo + gl;
        load_block_scaled<G, RMAX, B>(W, nrm2, dsc, keep, n, ld, lane, x, nx, dxs);
#pragma unroll
        for (int i = 0; i < B; ++i) dx[i] = false;
      }
      const int steps = (lmax + 1) >> 1;
      for (int s = 0; s < steps; ++s) {
        if (mine && s < nbk) {
          int qb = gl + s;
          if (qb >= nbk) qb -= nbk;
          const int Q = lo + h + qb;
          float y[B][RMAX], ny[B], dys[B];
          bool dy[B];
          load_block_scaled<G, RMAX, B>(W, nrm2, dsc, Q, n, ld, lane, y, ny, dys);
#pragma unroll
          for (int i = 0; i < B; ++i) dy[i] = false;
#pragma unroll
          for (int st = 0; st < B; ++st)
            rotate_scaled<G, RMAX, B>(x, y, nx, ny, dxs, dys, dx, dy, [](int i) { return i; },
                                      [st](int i) { return (i + st) % B; }, tol2, stop2, big, nrot);
          store_block_scaled<G, RMAX, B>(W, nrm2, dsc, Q, n, ld, lane, y, ny, dys, dy);
          // a long-kept block folds its scales in registers (as a store would)
#pragma unroll
          for (int i = 0; i < B; ++i)
            if (dxs[i] < 0x1p-12f || dxs[i] > 0x1p12f) {
#pragma unroll
              for (int k = 0; k < RMAX; ++k) x[i][k] *= dxs[i];
              dxs[i] = 1.f;
            }
        }
        __syncthreads();
      }
    }
    if (keep >= 0) store_block_scaled<G, RMAX, B>(W, nrm2, dsc, keep, n, ld, lane, x, nx, dxs, dx);
    if (lane == 0 && big) rot_flag[sweep] = __float_as_int(1.f);  // any group may set it
    __syncthreads();
    if (__int_as_float(rot_flag[sweep]) < stop) {
      sweeps = sweep + 1;
      break;
    }
  }
  // fold the remaining scales into the columns
  __syncthreads();
  for (int c = grp; c < n; c += ngrp) {
    const float dc = dsc[c];
    if (dc == 1.f) continue;
    float* col = W + c * ld + lane;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane + k * G < n) col[k * G] *= dc;
  }
  __syncthreads();
  return sweeps;
}

// Work-group reductions through a small shared scratch array (>= BLOCK/64 slots).
template <int BLOCK, typename T, typename Op>
__device__ T block_reduce(T v, T* scratch, Op op) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  T r = scratch[0];
  for (int i = 1; i < BLOCK / 64; ++i) r = op(r, scratch[i]);
  __syncthreads();
  return r;
}

}  // namespace wpcd
