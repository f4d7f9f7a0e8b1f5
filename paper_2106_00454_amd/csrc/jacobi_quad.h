// One-sided FP32 Jacobi in which a 16-lane row rotates the NB disjoint pairs
// of a stage at once and computes their NB angles once, each in one part of
// 16/NB lanes (Sec. 4.2, parallel cyclic-order Jacobi, over column blocks).
//
// The scaled-rotation iteration of onesided_jacobi_blocked_scaled (same skip
// test, same angle, shears and scale updates, same stopping rule), organised
// for fewer instructions per rotation:
// * a lane group is one 16-lane DPP row; it holds two blocks of NB columns
//   (P and Q, NB = 2 or 4) in registers and rotates the NB*NB cross pairs in
//   NB stages of NB disjoint pairs, pair i of stage s being
//   (x_i, y_(i+s) mod NB);
// * the NB dot products of a stage are reduced together: the row's halves
//   exchange partial sums (and for NB = 4 then its quarters), then each part
//   sums over its own lanes by a butterfly, so part i ends with pair i's dot
//   product, bitwise equal in all its lanes;
// * each lane then computes the angle of its part's pair: the NB angles of a
//   stage cost one instruction stream instead of NB, and no lane computes an
//   angle for another part;
// * the shear coefficients of the NB pairs go to every lane of the row by
//   row_newbcast; the shears run for every pair of a wavefront that rotates
//   any (a skipped pair has coefficient 0 and leaves its columns bitwise
//   unchanged), so the lane groups of a wavefront never diverge;
// * part i keeps the norm and scale of x_i for the whole step and those of
//   the y column it pairs with; after every stage the y states move one part
//   down the row (row_ror), so each part always holds the state of the
//   columns it rotates and no state is broadcast.
// NB = 4: 25 block pairs per step for n = 200, 49 steps (one barrier each),
// 8 wavefronts; NB = 2: 50 block pairs, 99 steps, 16 wavefronts.
#pragma once

#include "devutil.h"

namespace wpcd {

constexpr int kRowRor8 = 0x128;   // row_ror:8  (lane i reads lane i ^ 8 of its row)
constexpr int kRowRor12 = 0x12C;  // row_ror:12 (lane i reads lane (i + 4) mod 16 of its row)
template <int L>
__device__ __forceinline__ float row_bcast(float v) {  // row_newbcast:L (every lane reads lane L of its row)
  return dpp_f32<0x150 + L>(v);
}
template <int L>
__device__ __forceinline__ int row_bcast_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + L, 0xF, 0xF, false);
}

// Part q of each 16-lane row (16/NB lanes) receives the full sum over the
// row of v[q], bitwise equal in all lanes of the part.
template <int NB>
__device__ __forceinline__ float part_sums(const float (&v)[NB], int lane16) {
  static_assert(NB == 2 || NB == 4, "pairs per stage");
  const bool hi8 = (lane16 & 8) != 0;
  if constexpr (NB == 4) {
    const float k0 = hi8 ? v[2] : v[0], s0 = hi8 ? v[0] : v[2];
    const float k1 = hi8 ? v[3] : v[1], s1 = hi8 ? v[1] : v[3];
    const float a0 = k0 + dpp_f32<kRowRor8>(s0);  // lanes 0-7: pair 0, lanes 8-15: pair 2
    const float a1 = k1 + dpp_f32<kRowRor8>(s1);  // lanes 0-7: pair 1, lanes 8-15: pair 3
    const bool hi4 = (lane16 & 4) != 0;           // row_half_mirror pairs quarter 0 with 1 and 2 with 3
    const float k2 = hi4 ? a1 : a0, s2 = hi4 ? a0 : a1;
    float c = k2 + dpp_f32<kRowHalfMirror>(s2);
    c += dpp_f32<kQuadXor1>(c);
    c += dpp_f32<kQuadXor2>(c);
    return c;
  } else {
    const float k0 = hi8 ? v[1] : v[0], s0 = hi8 ? v[0] : v[1];
    float c = k0 + dpp_f32<kRowRor8>(s0);  // lanes 0-7: pair 0, lanes 8-15: pair 1
    c += dpp_f32<kRowHalfMirror>(c);       // lane i + lane 7-i of each half
    c += dpp_f32<kQuadXor2>(c);
    c += dpp_f32<kQuadXor1>(c);
    return c;
  }
}

// Columns blk*NB .. blk*NB+NB-1 of W into registers (row lane16 + 16 k of
// each); rows below (RMAX-1)*16 unguarded, the last chunk read in full and
// masked.
template <int NB, int RMAX>
__device__ __forceinline__ void part_load(const float* W, int blk, int n, int ld, int lane16,
                                          float (&x)[NB][RMAX]) {
  const bool last_ok = lane16 + (RMAX - 1) * 16 < n;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const float* col = W + (blk * NB + i) * ld + lane16;
#pragma unroll
    for (int k = 0; k < RMAX - 1; ++k) x[i][k] = col[k * 16];
    const float v = col[(RMAX - 1) * 16];
    x[i][RMAX - 1] = last_ok ? v : 0.f;
  }
}

// Stores the columns of a block whose flag has bit 0 (rotated), folding the
// scale into the column first when the flag has bit 1 (scale outside
// [2^-12, 2^12]); the first lane of part i writes column i's norm and scale.
template <int NB, int RMAX>
__device__ __forceinline__ void part_store(float* W, float* nrm2, float* dsc, int blk, int n, int ld, int lane16,
                                           float (&x)[NB][RMAX], const int (&flag)[NB], const float (&scale)[NB],
                                           float nrm_own, float dsc_own, int flag_own) {
  constexpr int PL = 16 / NB;  // lanes per part
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int c = blk * NB + i;
    if (c >= n || !(flag[i] & 1)) continue;
    if (flag[i] & 2) {
#pragma unroll
      for (int k = 0; k < RMAX; ++k) x[i][k] *= scale[i];
    }
    float* col = W + c * ld + lane16;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane16 + k * 16 < n) col[k * 16] = x[i][k];
  }
  const int c = blk * NB + lane16 / PL;
  if (lane16 % PL == 0 && c < n && (flag_own & 1)) {
    nrm2[c] = nrm_own;
    dsc[c] = (flag_own & 2) ? 1.f : dsc_own;
  }
}

// row_newbcast of lane i * 16/NB (the first lane of part i) for i < NB
template <int NB>
__device__ __forceinline__ void part_bcast(float v, float (&out)[NB]) {
  out[0] = row_bcast<0>(v);
  if constexpr (NB == 2) {
    out[1] = row_bcast<8>(v);
  } else {
    out[1] = row_bcast<4>(v);
    out[2] = row_bcast<8>(v);
    out[3] = row_bcast<12>(v);
  }
}
template <int NB>
__device__ __forceinline__ void part_bcast_i(int v, int (&out)[NB]) {
  out[0] = row_bcast_i<0>(v);
  if constexpr (NB == 2) {
    out[1] = row_bcast_i<8>(v);
  } else {
    out[1] = row_bcast_i<4>(v);
    out[2] = row_bcast_i<8>(v);
    out[3] = row_bcast_i<12>(v);
  }
}

// The iteration.  W holds nb*NB columns (columns n .. nb*NB-1 zero, never
// rotated) with ld >= (RMAX-1)*16 rows, zero below n, and 16 spare floats
// after the last column; nrm2 and dsc hold nb*NB floats each.  BLOCK/16 lane
// groups.  Same return value and rot_flag protocol as
// onesided_jacobi_blocked_scaled; on return the scales are folded into W.
template <int BLOCK, int RMAX, int NB>
__device__ int onesided_jacobi_parts(float* W, int n, int ld, float tol, float stop, int max_sweeps, int* rot_flag,
                                     float* nrm2, float* dsc, int& nrot) {
  static_assert(NB == 2 || NB == 4, "pairs per stage");
  constexpr int G = 16;
  constexpr int PL = G / NB;                              // lanes per part
  constexpr int kShift = NB == 4 ? kRowRor12 : kRowRor8;  // lane i reads lane i + PL of its row
  constexpr int ngrp = BLOCK / G;
  const int nb = (n + NB - 1) / NB;
  const int nbp = (nb + 1) >> 1;
  const int nbe = nbp << 1;
  const int lane16 = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int q = lane16 / PL;  // this lane's part
  const float tol2 = tol * tol, stop2 = stop * stop;
  for (int c = threadIdx.x; c < nb * NB; c += BLOCK) {
    dsc[c] = 1.f;
    nrm2[c] = 0.f;  // stays 0 for the zero columns
  }
  int sweeps = max_sweeps + 1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    bool big = false;
    __syncthreads();
    // exact squared norms of the true columns at the start of the sweep
    for (int c = grp; c < n; c += ngrp) {
      const float* col = W + c * ld + lane16;
      float s2 = 0.f;
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < RMAX - 1 || lane16 + k * G < n) s2 = fmaf(col[k * G], col[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane16 == 0) nrm2[c] = s2 * dsc[c] * dsc[c];
    }
    __syncthreads();
    // the pairs inside each block (NB = 4: three stages of two disjoint
    // pairs; NB = 2: the one pair)
    for (int blk = grp; blk < nb; blk += ngrp) {
      float x[NB][RMAX], nx[NB], d[NB];
      bool dx[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) dx[i] = false;
      load_block_scaled<G, RMAX, NB>(W, nrm2, dsc, blk, n, ld, lane16, x, nx, d);
#pragma unroll
      for (int st = 0; st < NB - 1; ++st) {
        auto col = [st](int c) { return c == 0 ? 0 : 1 + (c - 1 + st) % (NB - 1); };
        rotate_scaled<G, RMAX, NB / 2>(x, x, nx, nx, d, d, dx, dx, [&](int i) { return col(i); },
                                       [&](int i) { return col(NB - 1 - i); }, tol2, stop2, big, nrot);
      }
      store_block_scaled<G, RMAX, NB>(W, nrm2, dsc, blk, n, ld, lane16, x, nx, d, dx);
    }
    __syncthreads();
    // cross pairs of the block pairs of each round-robin step
    for (int step = 0; step < nbe - 1; ++step) {
      for (int pr = grp; pr < nbp; pr += ngrp) {
        const int P = rr_index_nodiv(pr, step, nbe);
        const int Q = rr_index_nodiv(nbe - 1 - pr, step, nbe);
        if (P >= nb || Q >= nb) continue;  // the padding block of odd nb
        float x[NB][RMAX], y[NB][RMAX];
        part_load<NB, RMAX>(W, P, n, ld, lane16, x);
        part_load<NB, RMAX>(W, Q, n, ld, lane16, y);
        // part q: state of x_q and of the y column it pairs with
        float nxq = nrm2[P * NB + q], sxq = dsc[P * NB + q];
        float nyq = nrm2[Q * NB + q], syq = dsc[Q * NB + q];
        int fx = 0, fy = 0;  // rotated flags of those columns
#pragma unroll
        for (int st = 0; st < NB; ++st) {
          float part[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < RMAX; ++k) a = fmaf(x[i][k], y[(i + st) % NB][k], a);
            part[i] = a;
          }
          const float dot = part_sums<NB>(part, lane16);
          // angle of this part's pair (x_q, y_(q+st))
          const float pq = sxq * syq;
          const float g = dot * pq;
          const float al = nxq, be = nyq;
          const float ab = al * be, g2 = g * g;
          const bool rot = g2 > tol2 * ab;
          const float D = be - al;
          float t = copysignf(1.f, D) * (2.f * g) *
                    __builtin_amdgcn_rcpf(fabsf(D) + __builtin_amdgcn_sqrtf(fmaf(D, D, 4.f * g2)));
          t = rot ? t : 0.f;
          const float u = fmaf(t, t, 1.f);
          const float c = __builtin_amdgcn_rsqf(u);
          const float r = t * __builtin_amdgcn_rcpf(pq);
          const float bq = r * sxq * sxq, ap = r * syq * syq * c * c;
          nxq = fmaf(-t, g, al);
          nyq = fmaf(t, g, be);
          sxq = sxq * u * c;
          syq = c * syq;
          fx |= rot ? 1 : 0;
          fy |= rot ? 1 : 0;
          big = big || (rot && g2 > stop2 * ab);
          if (rot && lane16 % PL == 0) ++nrot;
          // the NB pairs' shears in every lane; a wavefront none of whose
          // pairs rotates skips them (the converging sweeps rotate few)
          if (__any(rot)) {
            float cb[NB], ca[NB];
            part_bcast<NB>(bq, cb);
            part_bcast<NB>(ap, ca);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              const int j = (i + st) % NB;
#pragma unroll
              for (int k = 0; k < RMAX; ++k) {
                y[j][k] = fmaf(cb[i], x[i][k], y[j][k]);
                x[i][k] = fmaf(-ca[i], y[j][k], x[i][k]);
              }
            }
          }
          // part q pairs with y_(q+st+1) next: take that state from part q+1
          nyq = dpp_f32<kShift>(nyq);
          syq = dpp_f32<kShift>(syq);
          fy = __builtin_amdgcn_update_dpp(0, fy, kShift, 0xF, 0xF, false);
        }
        // after NB moves part q holds y_q again; flags (bit 0 rotated, bit 1
        // scale to fold) and scales of all 2 NB columns in every lane
        const int gx = fx | ((sxq < 0x1p-12f || sxq > 0x1p12f) ? 2 : 0);
        const int gy = fy | ((syq < 0x1p-12f || syq > 0x1p12f) ? 2 : 0);
        int flx[NB], fly[NB];
        float scx[NB], scy[NB];
        part_bcast_i<NB>(gx, flx);
        part_bcast_i<NB>(gy, fly);
        part_bcast<NB>(sxq, scx);
        part_bcast<NB>(syq, scy);
        part_store<NB, RMAX>(W, nrm2, dsc, P, n, ld, lane16, x, flx, scx, nxq, sxq, gx);
        part_store<NB, RMAX>(W, nrm2, dsc, Q, n, ld, lane16, y, fly, scy, nyq, syq, gy);
      }
      __syncthreads();
    }
    if (big) rot_flag[sweep] = __float_as_int(1.f);  // any lane may set it
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
    float* col = W + c * ld + lane16;
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < RMAX - 1 || lane16 + k * G < n) col[k * G] *= dc;
  }
  __syncthreads();
  return sweeps;
}

}  // namespace wpcd
