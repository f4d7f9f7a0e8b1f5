// FP64 refinement of all eigenpairs produced by the FP32 eigensolver.
//
// One step (Ogita & Aishima, "Iterative refinement for symmetric eigenvalue
// decomposition", Japan J. Indust. Appl. Math. 35 (2018)) for X ~ eigenvectors
// of A = H0 + V in FP64:
//   Y = A X,  S = X^T Y,  G = X^T X,  R = I - G,  lam_i = S_ii / G_ii,
//   delta = 2 (|S - diag(lam)|_F + |A|_F |R|_F),
//   E_ij = (S_ij + lam_j R_ij)/(lam_j - lam_i)  if |lam_j - lam_i| > delta,
//   E_ij = R_ij / 2                              otherwise (and on i = j),
//   X <- X + X E.
// Eigenvalues closer than delta form clusters (maximal runs of consecutive
// gaps <= delta) that a Newton step cannot separate; the cluster kernel then
// solves the Rayleigh-Ritz problem X_c^T A X_c in FP64 for every cluster and
// rotates X_c onto its eigenvectors.  All clusters of an item are solved at
// once as one block-diagonal matrix by the one-sided Jacobi kernel core:
// columns of different blocks are exactly orthogonal, so no rotation mixes
// blocks.
//
// The four n x n products per step are dense FP64 contractions and run on the
// matrix cores (v_mfma_f64_16x16x4f64), one work-group per item walking its
// 64 x 64 output tiles; 16 x 16 blocks entirely beyond n are skipped.
#include <float.h>

#include "devutil.h"
#include "internal.h"

namespace wpcd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;   // 4 wavefronts
constexpr int kTM = 64;       // output tile
constexpr int kTK = 16;       // K chunk
constexpr int kLdT = kTM + 4; // LDS row stride of a staged tile (doubles)
constexpr int kChunk = 64;    // columns per Rayleigh-Ritz batch

// Stage a 64 x 16 operand tile into LDS as T[k*kLdT + i], element (i,k) = f(r0+i, k0+k)
// (zero outside [0,n) x [0,kn)).  KC: the source is contiguous along k.
template <bool KC, class F>
__device__ __forceinline__ void stage(double* T, int r0, int k0, int n_i, int n_k, const F& f) {
  const int tid = threadIdx.x;
  if (KC) {
    const int i = tid >> 2, kb = (tid & 3) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kb + j;
      T[k * kLdT + i] = (r0 + i < n_i && k0 + k < n_k) ? f(r0 + i, k0 + k) : 0.0;
    }
  } else {
    const int k = tid >> 4, ib = (tid & 15) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = ib + j;
      T[k * kLdT + i] = (r0 + i < n_i && k0 + k < n_k) ? f(r0 + i, k0 + k) : 0.0;
    }
  }
}

// acc = sum_k A(m0+i, k) B(k, c0+j) over one 64 x 64 output tile.
// A(i,k) = fa(i,k) for i < rows, k < K; B(k,j) = fb(j,k) for j < cols, k < K.
// Both functors take (output index, reduction index): for a row-major matrix M
// the A operand M is RowMajor (fa(i,k) = M[i][k]) and the B operand M is
// RowMajorT (fb(j,k) = M[k][j]); A = M^T is RowMajorT and B = M^T is RowMajor.
template <bool AKC, bool BKC, class FA, class FB>
__device__ void gemm_tile(double* As, double* Bs, int m0, int c0, int rows, int cols, int K, const FA& fa,
                          const FB& fb, d4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  bool live[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) live[bi][bj] = (m0 + wr + bi * 16 < rows) && (c0 + wc + bj * 16 < cols);
  for (int k0 = 0; k0 < K; k0 += kTK) {
    stage<AKC>(As, m0, k0, rows, K, fa);
    stage<BKC>(Bs, c0, k0, cols, K, fb);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) a[bi] = As[kr * kLdT + wr + bi * 16 + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[kr * kLdT + wc + bj * 16 + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          if (live[bi][bj]) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
}

// Visit the accumulator entries of a tile: g(row, col, value) for in-range entries.
// v_mfma_f64_16x16x4f64 leaves D[i][j] in lane j + 16*(i % 4), register i / 4
// (A[i][k] comes from lane i + 16k, B[k][j] from lane j + 16k).
template <class G>
__device__ __forceinline__ void tile_store(int m0, int c0, int rows, int cols, const d4 (&acc)[2][2], const G& g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = c0 + wc + bj * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + bi * 16 + (lane >> 4) + 4 * r;
        if (row < rows && col < cols) g(row, col, acc[bi][bj][r]);
      }
    }
}

struct HOp {  // A = V + diag(e0 per channel copy)
  const double* V;
  const double* e0;
  int n, N;
  __device__ double operator()(int i, int k) const {
    double h = V[(int64_t)i * n + k];
    if (i == k) h += e0[i % N];
    return h;
  }
};

template <typename XT>
struct RowMajor {  // element (r, c) of a row-major n x ld matrix
  const XT* p;
  int ld;
  __device__ double operator()(int r, int c) const { return (double)p[(int64_t)r * ld + c]; }
};
template <typename XT>
struct RowMajorT {  // transposed view: (i, k) -> M(k, i)
  const XT* p;
  int ld;
  __device__ double operator()(int i, int k) const { return (double)p[(int64_t)k * ld + i]; }
};

struct EOp {  // B(k, j) = E(k, j), passed as fb(j, k)
  const double* S;
  const double* G;
  const double* lam;  // LDS
  double delta;
  int n;
  __device__ double operator()(int j, int k) const {
    const double g = G[(int64_t)k * n + j];
    if (j == k) return 0.5 * (1.0 - g);
    const double d = lam[j] - lam[k];
    const double r = -g;
    if (fabs(d) > delta) return (S[(int64_t)k * n + j] + lam[j] * r) / d;
    return 0.5 * r;
  }
};

// ---------------------------------------------------------------------------
// Newton-type step: X (row-major, XT) -> Xout (row-major, FP64), lam -> eval,
// cluster starts -> cl.  Work-space per item: P1 | Y | S | G (4 n^2 doubles);
// X and Xout are either the caller's array (offset v_off) or P1.
template <typename XT>
__global__ __launch_bounds__(kBlock) void refine_step_kernel(const ItemDev* __restrict__ items,
                                                             const GridDev* __restrict__ grids,
                                                             const double* __restrict__ v64, const XT* xin,
                                                             int xin_ws, double* evec, int xout_ws,
                                                             double* __restrict__ eval, double* work,
                                                             int32_t* __restrict__ cl) {
  __shared__ double As[kTK * kLdT];
  __shared__ double Bs[kTK * kLdT];
  __shared__ double lam[kMaxN];
  __shared__ double scratch[kBlock / 64];
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  const GridDev g = grids[it.grid];
  const HOp H{v64 + it.v_off, g.e0, n, it.N};
  const int64_t nn = (int64_t)n * n;
  double* P1 = work + it.w_off;
  double* Y = P1 + nn;
  double* S = Y + nn;
  double* Gm = S + nn;
  const XT* X = xin_ws ? reinterpret_cast<const XT*>(P1) : (xin + it.v_off);
  double* Xo = xout_ws ? P1 : (evec + it.v_off);
  const int nt = (n + kTM - 1) / kTM;
  d4 acc[2][2];

  // Y = A X
  for (int tm = 0; tm < nt; ++tm)
    for (int tc = 0; tc < nt; ++tc) {
      gemm_tile<true, false>(As, Bs, tm * kTM, tc * kTM, n, n, n, H, RowMajorT<XT>{X, n}, acc);
      tile_store(tm * kTM, tc * kTM, n, n, acc, [&](int r, int c, double v) { Y[(int64_t)r * n + c] = v; });
    }
  __syncthreads();
  // S = X^T Y and G = X^T X (upper tiles only; mirrored on store)
  for (int tm = 0; tm < nt; ++tm)
    for (int tc = tm; tc < nt; ++tc) {
      gemm_tile<false, false>(As, Bs, tm * kTM, tc * kTM, n, n, n, RowMajorT<XT>{X, n}, RowMajorT<double>{Y, n},
                              acc);
      // upper triangle only, mirrored: one writer per symmetric pair (deterministic)
      tile_store(tm * kTM, tc * kTM, n, n, acc, [&](int r, int c, double v) {
        if (r > c) return;
        S[(int64_t)r * n + c] = v;
        S[(int64_t)c * n + r] = v;
      });
      gemm_tile<false, false>(As, Bs, tm * kTM, tc * kTM, n, n, n, RowMajorT<XT>{X, n}, RowMajorT<XT>{X, n}, acc);
      tile_store(tm * kTM, tc * kTM, n, n, acc, [&](int r, int c, double v) {
        if (r > c) return;
        Gm[(int64_t)r * n + c] = v;
        Gm[(int64_t)c * n + r] = v;
      });
    }
  __syncthreads();
  // Rayleigh quotients, Frobenius norms and the cluster threshold
  for (int i = threadIdx.x; i < n; i += kBlock) lam[i] = S[(int64_t)i * n + i] / Gm[(int64_t)i * n + i];
  __syncthreads();
  double s2 = 0.0, r2 = 0.0, a2 = 0.0;
  for (int64_t e = threadIdx.x; e < nn; e += kBlock) {
    const int r = (int)(e / n), c = (int)(e - (int64_t)r * n);
    const double sv = S[e] - (r == c ? lam[r] : 0.0);
    const double rv = (r == c ? 1.0 : 0.0) - Gm[e];
    const double av = H(r, c);
    s2 = fma(sv, sv, s2);
    r2 = fma(rv, rv, r2);
    a2 = fma(av, av, a2);
  }
  auto sum = [](double a, double b) { return a + b; };
  s2 = block_reduce<kBlock>(s2, scratch, sum);
  r2 = block_reduce<kBlock>(r2, scratch, sum);
  a2 = block_reduce<kBlock>(a2, scratch, sum);
  const double delta = 2.0 * (sqrt(s2) + sqrt(a2) * sqrt(r2));
  // cluster starts: maximal runs of consecutive eigenvalues with gaps <= delta
  if (threadIdx.x == 0) {
    int start = 0;
    int32_t* c = cl + it.e_off;
    c[0] = 0;
    for (int i = 1; i < n; ++i) {
      if (!(lam[i] - lam[i - 1] <= delta)) start = i;
      c[i] = start;
    }
  }
  // X <- X + X E
  for (int tm = 0; tm < nt; ++tm)
    for (int tc = 0; tc < nt; ++tc) {
      gemm_tile<true, false>(As, Bs, tm * kTM, tc * kTM, n, n, n, RowMajor<XT>{X, n}, EOp{S, Gm, lam, delta, n},
                             acc);
      tile_store(tm * kTM, tc * kTM, n, n, acc,
                 [&](int r, int c, double v) { Xo[(int64_t)r * n + c] = (double)X[(int64_t)r * n + c] + v; });
    }
  for (int i = threadIdx.x; i < n; i += kBlock) eval[it.e_off + i] = lam[i];
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz inside clusters, batched in chunks of whole clusters of at
// most kChunk columns.  X is row-major FP64 (in place).  Work-space: Z in the
// S region (n x T, row stride T), Q in the G region (T x T); T <= n, so both fit
// their n x n regions.
__global__ __launch_bounds__(kBlock) void refine_cluster_kernel(const ItemDev* __restrict__ items,
                                                                const GridDev* __restrict__ grids,
                                                                const double* __restrict__ v64, double* xbase,
                                                                int x_ws, double* __restrict__ eval, double* work,
                                                                const int32_t* __restrict__ cl,
                                                                int32_t* __restrict__ status) {
  __shared__ double As[kTK * kLdT];
  __shared__ double Bs[kTK * kLdT];
  __shared__ double W[kChunk * (kChunk | 1)];
  __shared__ double shift[kChunk];
  __shared__ double nrm[kChunk];
  __shared__ int cols[kChunk];
  __shared__ int blk[kChunk];  // first chunk position of each column's cluster
  __shared__ int rot_flag[64];
  __shared__ int s_chunk_len, s_next, s_fail;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  const GridDev g = grids[it.grid];
  const HOp H{v64 + it.v_off, g.e0, n, it.N};
  const int64_t nn = (int64_t)n * n;
  double* P1 = work + it.w_off;
  double* Z = P1 + 2 * nn;  // S region
  double* Q = P1 + 3 * nn;  // G region
  double* X = x_ws ? P1 : (xbase + it.v_off);
  const int32_t* c = cl + it.e_off;
  double* ev = eval + it.e_off;
  constexpr int ldw = kChunk | 1;
  if (threadIdx.x == 0) {
    s_next = 0;
    s_fail = 0;
  }
  __syncthreads();
  while (true) {
    // gather the next chunk of whole clusters (size >= 2)
    if (threadIdx.x == 0) {
      int i = s_next, len = 0;
      while (i < n) {
        int j = i + 1;
        while (j < n && c[j] == i) ++j;
        const int m = j - i;
        if (m >= 2) {
          if (m > kChunk) {  // too large for one Rayleigh-Ritz batch: leave it refined by Newton only
            s_fail = 1;
          } else if (len + m > kChunk) {
            break;
          } else {
            for (int q = 0; q < m; ++q) {
              cols[len + q] = i + q;
              blk[len + q] = len;
            }
            len += m;
          }
        }
        i = j;
      }
      s_next = i;
      s_chunk_len = len;
    }
    __syncthreads();
    const int T = s_chunk_len;
    if (T == 0) break;
    d4 acc[2][2];
    // Z = A X[:, cols]   (n x T)
    const int nt = (n + kTM - 1) / kTM;
    auto xcols = [&](int j, int k) { return X[(int64_t)k * n + cols[j]]; };  // B(k, j) = X(k, cols[j])
    for (int tm = 0; tm < nt; ++tm) {
      gemm_tile<true, false>(As, Bs, tm * kTM, 0, n, T, n, H, xcols, acc);
      tile_store(tm * kTM, 0, n, T, acc, [&](int r, int cc, double v) { Z[(int64_t)r * T + cc] = v; });
    }
    __syncthreads();
    // S_c = X[:, cols]^T Z, kept block-diagonal, into W (column-major)
    {
      auto xt = [&](int i, int k) { return X[(int64_t)k * n + cols[i]]; };  // A(i, k) = X(k, cols[i])
      auto zc = [&](int j, int k) { return Z[(int64_t)k * T + j]; };
      gemm_tile<false, false>(As, Bs, 0, 0, T, T, n, xt, zc, acc);
      tile_store(0, 0, T, T, acc, [&](int r, int cc, double v) { W[cc * ldw + r] = (blk[r] == blk[cc]) ? v : 0.0; });
    }
    if (threadIdx.x < 64) rot_flag[threadIdx.x] = 0;
    __syncthreads();
    // per-block Gershgorin shift making every block positive definite
    for (int j = threadIdx.x; j < T; j += kBlock) {
      if (blk[j] != j) continue;  // one thread per block, at its first column
      int e = j + 1;
      while (e < T && blk[e] == j) ++e;
      double lo = DBL_MAX, hi = -DBL_MAX;
      for (int q = j; q < e; ++q) {
        double s = 0.0;
        for (int r = j; r < e; ++r)
          if (r != q) s += fabs(W[q * ldw + r]);
        const double d = W[q * ldw + q];
        lo = fmin(lo, d - s);
        hi = fmax(hi, d + s);
      }
      const double sh = (lo < 0.0 ? -lo : 0.0) + 0.05 * (hi - lo) + DBL_MIN;
      for (int q = j; q < e; ++q) shift[q] = sh;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < T; j += kBlock) W[j * ldw + j] += shift[j];
    __syncthreads();
    const int sw = onesided_jacobi_lds<double, kBlock, 4, 16>(W, T, ldw, 1e-15, 40, rot_flag);
    if (sw > 40 && threadIdx.x == 0) s_fail = 1;
    for (int j = threadIdx.x; j < T; j += kBlock) {
      double s2 = 0.0;
      for (int r = 0; r < T; ++r) s2 = fma(W[j * ldw + r], W[j * ldw + r], s2);
      nrm[j] = sqrt(s2);
    }
    __syncthreads();
    // Q(:, rank) = w_j/|w_j| with the rank taken inside the block; eigenvalue |w_j| - shift
    for (int j = threadIdx.x; j < T; j += kBlock) {
      const int b0 = blk[j];
      const double lj = nrm[j] - shift[j];
      int rank = b0;
      for (int q = b0; q < T && blk[q] == b0; ++q) {
        const double lq = nrm[q] - shift[q];
        rank += (lq < lj || (lq == lj && q < j)) ? 1 : 0;
      }
      const double inv = 1.0 / nrm[j];
      for (int r = 0; r < T; ++r) Q[(int64_t)r * T + rank] = W[j * ldw + r] * inv;
      ev[cols[rank]] = lj;
    }
    __syncthreads();
    // X[:, cols] <- X[:, cols] Q, through Z as staging
    auto xa = [&](int i, int k) { return X[(int64_t)i * n + cols[k]]; };  // A(i, k) = X(i, cols[k])
    auto qb = [&](int j, int k) { return Q[(int64_t)k * T + j]; };
    for (int tm = 0; tm < nt; ++tm) {
      gemm_tile<false, false>(As, Bs, tm * kTM, 0, n, T, T, xa, qb, acc);
      tile_store(tm * kTM, 0, n, T, acc, [&](int r, int cc, double v) { Z[(int64_t)r * T + cc] = v; });
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < (int64_t)n * T; e += kBlock) {
      const int r = (int)(e / T), cc = (int)(e - (int64_t)r * T);
      X[(int64_t)r * n + cols[cc]] = Z[(int64_t)r * T + cc];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && s_fail && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// Final pass: copy X from the work-space when the last step left it there, and
// check the eigenvalues are ascending and finite.
__global__ __launch_bounds__(kBlock) void refine_finish_kernel(const ItemDev* __restrict__ items, double* evec,
                                                               int x_ws, const double* work,
                                                               const double* __restrict__ eval,
                                                               int32_t* __restrict__ status) {
  __shared__ int bad;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (x_ws) {
    const double* src = work + it.w_off;
    double* dst = evec + it.v_off;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kBlock) dst[e] = src[e];
  }
  const double* ev = eval + it.e_off;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    if (!isfinite(ev[i]) || (i > 0 && ev[i] < ev[i - 1])) bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

}  // namespace

hipError_t launch_refine(const ItemDev* items, int n_items, const GridDev* grids, const double* v64,
                         const float* x32, double* evec, double* eval, double* work, int32_t* cl, int32_t* status,
                         int steps, hipStream_t s) {
  // X ping-pongs between the caller's evec (ws = 0) and the work-space P1 (ws = 1)
  int cur_ws = 0;
  for (int st = 0; st < steps; ++st) {
    const int out_ws = (st == 0) ? 0 : 1 - cur_ws;
    if (st == 0)
      hipLaunchKernelGGL(refine_step_kernel<float>, dim3(n_items), dim3(kBlock), 0, s, items, grids, v64, x32, 0,
                         evec, out_ws, eval, work, cl);
    else
      hipLaunchKernelGGL(refine_step_kernel<double>, dim3(n_items), dim3(kBlock), 0, s, items, grids, v64,
                         (const double*)evec, cur_ws, evec, out_ws, eval, work, cl);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(refine_cluster_kernel, dim3(n_items), dim3(kBlock), 0, s, items, grids, v64, evec, out_ws,
                       eval, work, cl, status);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    cur_ws = out_ws;
  }
  hipLaunchKernelGGL(refine_finish_kernel, dim3(n_items), dim3(kBlock), 0, s, items, evec, cur_ws, work, eval,
                     status);
  return hipGetLastError();
}

}  // namespace wpcd
