// Block one-sided Jacobi with W in device memory (Sec. 3.1, H = C D C^T;
// Sec. 4.2, parallel cyclic-order Jacobi): FP32 for mixed-path items too large
// for LDS (n > 200), FP64 for every item of the plain path.
#include "jacobi_common.h"

namespace wpcd {
namespace {

// ---------------------------------------------------------- device-memory path
// Items too large for LDS (and every item of the plain FP64 path) keep W
// (n x n, column-major) in their device work-space and run a block Jacobi
// over column blocks of BW columns, one kernel launch per stage of the sweep so
// that the blocks of one item are spread over many compute units:
//   gjac_init:   W = H + sigma I (Gershgorin sigma), per-item state cleared;
//   gjac_block:  INTRA=true  -- one work-group per block rotates all pairs
//                               inside it (circle ordering over BW columns);
//                INTRA=false -- one work-group per block pair of round-robin
//                               step `step` rotates the BW*BW cross pairs in
//                               BW stages of BW disjoint pairs;
//                both stage the 2*BW (or BW) columns in LDS and write them back;
//   gjac_finish: column norms, eigenvalues, rank sort and outputs.
// A sweep is one INTRA launch plus the round-robin steps over blocks, so every
// column pair is rotated once per sweep.  Each launch first reads the previous
// sweep's largest rotated |w_p.w_q|/(|w_p||w_q|) (kept per item, atomically
// maxed as float bits) and does nothing once the item has converged, so the
// host can enqueue all sweeps without waiting.
template <typename T>
struct GJacState {
  T sigma;
  float stop;          // the iteration ends after a sweep whose largest rotated pair was below this
  int32_t pad[2];
  int32_t rotmax[64];  // per sweep, float bits of the largest rotated pair
};

template <typename T>
__device__ __forceinline__ GJacState<T>* gjac_state(double* work, const ItemDev& it) {
  // after W (n*n elements of T), 16-byte aligned, inside the 6 n^2 doubles
  const int64_t wbytes = ((int64_t)it.n * it.n * (int64_t)sizeof(T) + 15) & ~(int64_t)15;
  return reinterpret_cast<GJacState<T>*>(reinterpret_cast<char*>(work + it.w_off) + wbytes);
}

template <typename T>
__device__ __forceinline__ bool gjac_converged(const GJacState<T>* st, int sweep) {
  return sweep > 0 && __int_as_float(__atomic_load_n(&st->rotmax[sweep - 1], __ATOMIC_RELAXED)) < st->stop;
}

template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void gjac_init_kernel(const ItemDev* __restrict__ items,
                                                          const int32_t* __restrict__ sel,
                                                          const GridDev* __restrict__ grids,
                                                          const double* __restrict__ v64, double* work,
                                                          float stop, const int32_t* __restrict__ ref,
                                                          const float* __restrict__ x32) {
  __shared__ T scratch[BLOCK / 64];
  const int item = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  const ItemDev it = items[item];
  const int n = it.n, N = it.N;
  const GridDev g = grids[it.grid];
  const double* V = v64 + it.v_off;
  T* W = reinterpret_cast<T*>(work + it.w_off);
  GJacState<T>* st = gjac_state<T>(work, it);
  // Columns of B = H + sigma I in descending order of their norms, as in the
  // LDS kernel (column j of W is column perm[j] of B): first pass over V for
  // the Gershgorin bounds and |H e_c|^2, H_cc; second pass writes W.
  __shared__ T key[kMaxN];
  __shared__ T dg[kMaxN];
  __shared__ int perm[kMaxN];
  constexpr int G = 16;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  T lo = T(DBL_MAX), hi = T(-DBL_MAX);
  for (int c = grp; c < n; c += BLOCK / G) {
    T off = 0, h2 = 0, d = 0;
    for (int r = lane; r < n; r += G) {
      double h = V[(int64_t)c * n + r];
      if (r == c) h += g.e0[r % N];
      const T ht = (T)h;
      h2 = fma(ht, ht, h2);
      if (r == c) d = ht;
      else off += fabs(ht);
    }
    off = group_sum<G>(off);
    h2 = group_sum<G>(h2);
    d = group_sum<G>(d);
    lo = fmin(lo, d - off);
    hi = fmax(hi, d + off);
    if (lane == 0) {
      key[c] = h2;
      dg[c] = d;
    }
  }
  lo = block_reduce<BLOCK>(lo, scratch, MinOp<T>());
  hi = block_reduce<BLOCK>(hi, scratch, MaxOp<T>());
  const T sigma = (lo < T(0) ? -lo : T(0)) + T(0.05) * (hi - lo);
  const int rid = ref ? ref[item] : -1;
  if (rid >= 0) {
    // warm start: W = B Q0 = H Q0 + sigma Q0, with H Q0 (column-major FP32 in
    // this item's x32) and Q0 (the reference's eigenvectors, descending,
    // column-major floats in the reference's work-space) prepared by
    // launch_jacobi_warm_prep
    const float* Y0 = x32 + it.v_off;
    const float* Q0 = reinterpret_cast<const float*>(work + items[rid].w_off);
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = threadIdx.x; e < nn; e += BLOCK) W[e] = (T)fmaf((float)sigma, Q0[e], Y0[e]);
    for (int i = threadIdx.x; i < 64; i += BLOCK) st->rotmax[i] = 0;
    if (threadIdx.x == 0) {
      st->sigma = sigma;
      st->stop = stop;
    }
    return;
  }
  // a NaN key (NaN in V) ranks last, so the ranks stay a permutation (the
  // item is flagged by the finish kernel)
  for (int c = threadIdx.x; c < n; c += BLOCK) {
    const T kc = key[c] + sigma * (T(2) * dg[c] + sigma);
    key[c] = kc == kc ? kc : T(-INFINITY);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += BLOCK) {
    const T kc = key[c];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += (key[q] > kc || (key[q] == kc && q < c)) ? 1 : 0;
    perm[rank] = c;
  }
  __syncthreads();
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += BLOCK) {
    const int j = (int)(e / n), r = (int)(e - (int64_t)j * n);
    const int c = perm[j];
    double h = V[(int64_t)c * n + r];
    if (r == c) h += g.e0[r % N];
    T w = (T)h;
    if (r == c) w += sigma;
    W[e] = w;
  }
  for (int i = threadIdx.x; i < 64; i += BLOCK) st->rotmax[i] = 0;
  if (threadIdx.x == 0) {
    st->sigma = sigma;
    st->stop = stop;
  }
}

// LDS column stride of the block kernels: the smallest ld >= n with
// ld = G (mod 2G) for G < 64 (the 64/G lane groups of a wavefront, each
// reading G consecutive rows of its own column, start on distinct bank
// ranges when their columns are consecutive) and ld = 0 (mod 64) for G = 64.
template <int G>
__host__ __device__ constexpr int gjac_ld(int n) {
  return G >= 64 ? n + (64 - n % 64) % 64 : n + ((G - n % (2 * G)) % (2 * G) + 2 * G) % (2 * G);
}

// Rotates the column pair (p, q) held in LDS by a lane group of G, with the
// squared norms np, nq of the staged columns tracked in LDS (one dot product
// per pair; |w_p'|^2 = |w_p|^2 - t w_p.w_q, |w_q'|^2 = |w_q|^2 + t w_p.w_q).
template <typename T, int G, int RMAX>
__device__ __forceinline__ void lds_pair_rotate(T* wp, T* wq, T* np, T* nq, int n, int lane, T tol, T& rmax) {
  T xp[RMAX], xq[RMAX];
  T ga = T(0);
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    const int r = lane + k * G;
    const T a = r < n ? wp[r] : T(0), b = r < n ? wq[r] : T(0);
    xp[k] = a;
    xq[k] = b;
    ga = fma(a, b, ga);
  }
  ga = group_sum<G>(ga);
  const T al = *np, be = *nq;
  const T nab = sqrt(al * be);
  if (fabs(ga) > tol * nab) {
    const T zeta = (be - al) / (T(2) * ga);
    const T t = copysign(T(1), zeta) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
    const T c = T(1) / sqrt(T(1) + t * t);
    const T s = c * t;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
      const int r = lane + k * G;
      if (r < n) {
        wp[r] = c * xp[k] - s * xq[k];
        wq[r] = s * xp[k] + c * xq[k];
      }
    }
    if (lane == 0) {
      *np = al - t * ga;
      *nq = be + t * ga;
    }
    const T rel = fabs(ga) / nab;
    rmax = rel > rmax ? rel : rmax;
  }
}

template <typename T, int BW, int G, int RMAX, bool INTRA>
__global__ __launch_bounds__(BW * G) void gjac_block_kernel(const ItemDev* __restrict__ items,
                                                            const int32_t* __restrict__ sel, double* work,
                                                            int sweep, int step, T tol) {
  extern __shared__ char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);
  __shared__ int any_rot;
  const int item = sel ? sel[blockIdx.y] : (int)blockIdx.y;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nb = (n + BW - 1) / BW, nbp = (nb + 1) >> 1, nbe = nbp << 1;
  int blk[2];
  int nblk;
  if (INTRA) {
    if ((int)blockIdx.x >= nb) return;
    blk[0] = blockIdx.x;
    nblk = 1;
  } else {
    if (step >= nbe - 1 || (int)blockIdx.x >= nbp) return;
    blk[0] = rr_index(blockIdx.x, step, nbe);
    blk[1] = rr_index(nbe - 1 - blockIdx.x, step, nbe);
    if (blk[0] >= nb || blk[1] >= nb) return;  // the padding block of odd nb
    nblk = 2;
  }
  T* W = reinterpret_cast<T*>(work + it.w_off);
  GJacState<T>* st = gjac_state<T>(work, it);
  if (gjac_converged(st, sweep)) return;
  const int ld = gjac_ld<G>(n);
  // stage the columns (absent columns beyond n are zero and never written back)
  for (int b = 0; b < nblk; ++b)
    for (int j = threadIdx.y; j < BW; j += blockDim.y) {
      const int c = blk[b] * BW + j;
      T* dst = L + (b * BW + j) * ld;
      for (int r = threadIdx.x; r < n; r += G) dst[r] = c < n ? W[(int64_t)c * n + r] : T(0);
    }
  if (threadIdx.x == 0 && threadIdx.y == 0) any_rot = 0;
  __syncthreads();
  const int lane = threadIdx.x, grp = threadIdx.y;
  // exact squared norms of the staged columns (tracked through the stages)
  __shared__ T cn[2 * BW];
  for (int j = grp; j < nblk * BW; j += BW) {
    const T* col = L + j * ld;
    T s2 = T(0);
    for (int r = lane; r < n; r += G) s2 = fma(col[r], col[r], s2);
    s2 = group_sum<G>(s2);
    if (lane == 0) cn[j] = s2;
  }
  __syncthreads();
  T rmax = T(0);
  if (INTRA) {
    // circle ordering over the BW columns: BW-1 stages of BW/2 pairs
    for (int s = 0; s < BW - 1; ++s) {
      if (grp < BW / 2) {
        auto col = [s](int q) { return q == 0 ? 0 : 1 + (q - 1 + s) % (BW - 1); };
        const int a = col(grp), b = col(BW - 1 - grp);
        lds_pair_rotate<T, G, RMAX>(L + a * ld, L + b * ld, cn + a, cn + b, n, lane, tol, rmax);
      }
      __syncthreads();
    }
  } else {
    // cross pairs: stage s pairs column i of the first block with column
    // (i + s) mod BW of the second
    for (int s = 0; s < BW; ++s) {
      const int b = BW + (grp + s) % BW;
      lds_pair_rotate<T, G, RMAX>(L + grp * ld, L + b * ld, cn + grp, cn + b, n, lane, tol, rmax);
      __syncthreads();
    }
  }
  if (lane == 0 && rmax > T(0)) any_rot = 1;
  __syncthreads();
  if (!any_rot) return;  // nothing changed: W is already current
  for (int b = 0; b < nblk; ++b)
    for (int j = threadIdx.y; j < BW; j += blockDim.y) {
      const int c = blk[b] * BW + j;
      if (c >= n) continue;
      const T* src = L + (b * BW + j) * ld;
      for (int r = threadIdx.x; r < n; r += G) W[(int64_t)c * n + r] = src[r];
    }
  if (lane == 0 && rmax > T(0)) atomicMax(&st->rotmax[sweep], __float_as_int((float)rmax));
}

// flag[sweep] = 1 when every item of the launch has converged after sweep
// (its largest rotated pair of that sweep below its stopping threshold; an
// item converged earlier rotated nothing), else 0.  One work-group.
template <typename T>
__global__ __launch_bounds__(256) void gjac_flag_kernel(const ItemDev* __restrict__ items,
                                                        const int32_t* __restrict__ sel, int n_sel, double* work,
                                                        int sweep, int32_t* flag) {
  __shared__ int open;
  if (threadIdx.x == 0) open = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n_sel; i += blockDim.x) {
    const GJacState<T>* st = gjac_state<T>(work, items[sel ? sel[i] : i]);
    if (!(__int_as_float(st->rotmax[sweep]) < st->stop)) open = 1;  // NaN counts as not converged
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag + sweep, open ? 0 : 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Norms, eigenvalues and sorted outputs.  T = double: eigenvalues as Rayleigh
// quotients v^T H v / v^T v of v = w/|w| (exact for a diagonal H, free of the
// shift's rounding), eigenvectors to the caller's FP64 array.  T = float:
// eigenvalues |w| - sigma and FP32 eigenvectors in the row-major x32.
template <typename T, int BLOCK, int G>
__global__ __launch_bounds__(BLOCK) void gjac_finish_kernel(const ItemDev* __restrict__ items,
                                                            const int32_t* __restrict__ sel,
                                                            const GridDev* __restrict__ grids,
                                                            const double* __restrict__ v64, double* work,
                                                            double* __restrict__ evec, float* __restrict__ x32,
                                                            double* __restrict__ eval, int32_t* __restrict__ status,
                                                            int max_sweeps, T tol) {
  __shared__ int bad;
  __shared__ int rank_of[kMaxN];
  __shared__ double rq[kMaxN];
  __shared__ double nrm[kMaxN];
  const int item = sel ? sel[blockIdx.x] : (int)blockIdx.x;
  const ItemDev it = items[item];
  const int n = it.n;
  const T* W = reinterpret_cast<const T*>(work + it.w_off);
  const GJacState<T>* st = gjac_state<T>(work, it);
  const T sigma = st->sigma;
  int sweeps = max_sweeps + 1;
  for (int s = 0; s < max_sweeps; ++s)
    if (__int_as_float(st->rotmax[s]) < st->stop) {
      sweeps = s + 1;
      break;
    }
  if (threadIdx.x == 0) bad = 0;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  if constexpr (sizeof(T) == 8) {
    // FP64: normalise the columns in place (v = w/|w| by division, so an
    // unrotated column is an exact unit vector); the Rayleigh quotients, the
    // sort and the outputs follow in launch_rayleigh_f64
    T* Wm = reinterpret_cast<T*>(work + it.w_off);
    for (int c = grp; c < n; c += ngrp) {
      T* col = Wm + (int64_t)c * n;
      T s2 = 0;
      for (int r = lane; r < n; r += G) s2 = fma(col[r], col[r], s2);
      const T nc = sqrt(group_sum<G>(s2));
      if (!(nc > 0.0) || !isfinite(nc)) {
        if (lane == 0) bad = 1;
        continue;
      }
      for (int r = lane; r < n; r += G) col[r] = col[r] / nc;
    }
    __syncthreads();
  } else {
    for (int c = grp; c < n; c += ngrp) {
      const T* col = W + (int64_t)c * n;
      T s2 = 0;
      for (int r = lane; r < n; r += G) s2 = fma(col[r], col[r], s2);
      const T nc = sqrt(group_sum<G>(s2));
      if (lane == 0) {
        nrm[c] = (double)nc;
        rq[c] = (double)nc - (double)sigma;
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
      if (!(nc > 0.0) || !isfinite(nc)) {
        if (lane == 0) bad = 1;
        continue;
      }
      const int rank = rank_of[c];
      const T* col = W + (int64_t)c * n;
      float* X = x32 + it.v_off;
      for (int r = lane; r < n; r += G) X[(int64_t)r * n + rank] = (float)col[r] / (float)nc;
    }
    __syncthreads();
    double* ev = eval + it.e_off;
    for (int c = threadIdx.x; c < n; c += BLOCK) ev[rank_of[c]] = rq[c];
  }
  if (threadIdx.x == 0)
    status[item] = bad ? WPCD_ERR_NUMERIC : (sweeps > max_sweeps ? WPCD_ERR_NOCONV : sweeps);
}

// Host side: init, up to max_sweeps x (INTRA + round-robin steps), finish;
// with feedback the sweeps stop kJacLookahead sweeps after the first one
// that left every item converged.
template <typename T, int BW, int G, int RMAX>
hipError_t gjac_run(const ItemDev* items, const int32_t* sel, int n_sel, int max_n, const GridDev* grids,
                    const double* v64, double* work, double* evec, float* x32, double* eval, int32_t* status,
                    int max_sweeps, T tol, float stop, const int32_t* ref, JacFeedback* fb, hipStream_t s) {
  static_assert(BW * G <= 1024, "block size");
  if (max_n > RMAX * G) return hipErrorInvalidValue;
  const size_t lds = (size_t)2 * BW * gjac_ld<G>(max_n) * sizeof(T);
  if (lds + 1024 > 160 * 1024) return hipErrorInvalidValue;  // static LDS: flag, staged-column norms
  auto intra = gjac_block_kernel<T, BW, G, RMAX, true>;
  auto cross = gjac_block_kernel<T, BW, G, RMAX, false>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(intra),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(cross), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (e != hipSuccess) return e;
  const int nb = (max_n + BW - 1) / BW, nbp = (nb + 1) >> 1, nbe = nbp << 1;
  // feedback only outside stream capture (a captured sequence cannot wait)
  bool look = fb != nullptr && fb->flag != nullptr;
  if (look) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    look = cs == hipStreamCaptureStatusNone;
  }
  int32_t* dflag = nullptr;
  if (look) {
    e = hipHostGetDevicePointer((void**)&dflag, fb->flag, 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gjac_init_kernel<T, 1024>), dim3(n_sel), dim3(1024), 0, s, items, sel, grids, v64, work,
                     stop, ref, x32);
  int64_t launches = 2, sweeps = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    hipLaunchKernelGGL(intra, dim3(nb, n_sel), dim3(G, BW), lds, s, items, sel, work, sw, 0, tol);
    for (int step = 0; step < nbe - 1; ++step)
      hipLaunchKernelGGL(cross, dim3(nbp, n_sel), dim3(G, BW), lds, s, items, sel, work, sw, step, tol);
    launches += nbe;
    ++sweeps;
    if (!look) continue;
    hipLaunchKernelGGL(gjac_flag_kernel<T>, dim3(1), dim3(256), 0, s, items, sel, n_sel, work, sw, dflag);
    ++launches;
    e = hipEventRecord(fb->ev[sw % kJacFbEvents], s);
    if (e != hipSuccess) return e;
    if (sw >= kJacLookahead) {
      // the device still has kJacLookahead sweeps queued while the host waits
      e = hipEventSynchronize(fb->ev[(sw - kJacLookahead) % kJacFbEvents]);
      if (e != hipSuccess) return e;
      if (__atomic_load_n(fb->flag + (sw - kJacLookahead), __ATOMIC_ACQUIRE) == 1) break;
    }
  }
  if (fb != nullptr) {
    fb->launches += launches;
    fb->sweeps += sweeps;
  }
  hipLaunchKernelGGL((gjac_finish_kernel<T, 1024, 16>), dim3(n_sel), dim3(1024), 0, s, items, sel, grids, v64, work,
                     evec, x32, eval, status, max_sweeps, tol);
  if (sizeof(T) == 8) {
    if (sel) return hipErrorInvalidValue;  // the FP64 path runs on whole batches
    return launch_rayleigh_f64(items, n_sel, max_n, grids, v64, work, evec, eval, status, s);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t jac_feedback_create(JacFeedback& f) {
  hipError_t e = hipHostMalloc((void**)&f.flag, 64 * sizeof(int32_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    f.flag = nullptr;
    return e;
  }
  for (int i = 0; i < 64; ++i) f.flag[i] = 0;
  for (int i = 0; i < kJacFbEvents && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&f.ev[i], hipEventDisableTiming);
  if (e != hipSuccess) jac_feedback_destroy(f);
  return e;
}

void jac_feedback_destroy(JacFeedback& f) {
  for (int i = 0; i < kJacFbEvents; ++i) {
    if (f.ev[i]) hipEventDestroy(f.ev[i]);
    f.ev[i] = nullptr;
  }
  if (f.flag) hipHostFree(f.flag);
  f.flag = nullptr;
}

hipError_t launch_jacobi_global(int mixed, const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                const GridDev* grids, const double* v64, double* work, double* evec, float* x32,
                                double* eval, int32_t* status, int max_sweeps, double tol, double stop,
                                const int32_t* ref, JacFeedback* fb, hipStream_t s) {
  if (max_n > kMaxN || max_sweeps > 64) return hipErrorInvalidValue;
  if (n_sel == 0) return hipSuccess;
  // block width: two blocks of the largest item fill at most 160 KiB of LDS;
  // lane groups of G rows x RMAX rows per lane cover n
  if (mixed) {
    const float t = (float)tol;
    if (max_n <= 304)
      return gjac_run<float, 64, 16, 19>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                         max_sweeps, t, (float)stop, ref, fb, s);
    if (max_n <= 608)
      return gjac_run<float, 32, 32, 19>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                         max_sweeps, t, (float)stop, ref, fb, s);
    return gjac_run<float, 16, 64, 19>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                       max_sweeps, t, (float)stop, ref, fb, s);
  }
  if (max_n <= 144)
    return gjac_run<double, 64, 16, 9>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                       max_sweeps, tol, (float)stop, nullptr, fb, s);
  if (max_n <= 288)
    return gjac_run<double, 32, 32, 9>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                       max_sweeps, tol, (float)stop, nullptr, fb, s);
  if (max_n <= 576)
    return gjac_run<double, 16, 64, 9>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status,
                                        max_sweeps, tol, (float)stop, nullptr, fb, s);
  return gjac_run<double, 8, 64, 19>(items, sel, n_sel, max_n, grids, v64, work, evec, x32, eval, status, max_sweeps,
                                     tol, (float)stop, nullptr, fb, s);
}

}  // namespace wpcd
