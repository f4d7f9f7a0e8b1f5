// FP64 refinement of all eigenpairs produced by the FP32 eigensolver.
//
// One Newton-type step (after Ogita & Aishima, "Iterative refinement for
// symmetric eigenvalue decomposition", Japan J. Indust. Appl. Math. 35 (2018))
// for X ~ eigenvectors of A = H0 + V, all in FP64:
//   Y = A X,  S = X^T Y,  G = X^T X,  R = I - G,  lam_i = S_ii / G_ii,
//   E_ij = (S_ij + lam_j R_ij)/(lam_j - lam_i),  E_ii = R_ii/2,
//   X <- X (I + E).
// The first-order update is only accurate where |E_ij| is small.  A pair is
// called close when c |S_ij + lam_j R_ij| >= |lam_j - lam_i| (or the same with
// lam_i in the numerator), i.e. when its predicted correction would reach 1/c,
// with c = 1000 in the first step and 100x more in each later one.  Close
// pairs take E_ij = R_ij/2 (orthogonalisation only) and every maximal index
// range spanned by close pairs (a chain) is solved exactly by Rayleigh-Ritz:
// with P = (I + E)[:, chain], X P spans the refined chain subspace and
// (X P)^T A (X P) = P^T S P, whose eigenvectors Q (FP64 one-sided Jacobi)
// rotate the chain: the update becomes X <- X M with M = I + E except
// M[:, chain] = P Q.  The chain block P^T S P is formed without the n x n x m
// product S P: with C the chain's columns, P = I_C + E_C and T = S_C +
// Lam E_C / 2 (n x m, Lam = diag(lam)), V = P^T T gives
//   P^T S P = V + V^T - T_C - T_C^T + S_CC + E_C^T (S - Lam) E_C,
// where T_C, S_CC are the rows C of T and S_C.  S - Lam is of the order of the
// error of X (about 1e-7 |A| from FP32 vectors) and so is E_C off the close
// pairs (|E| < 1/c there), so the last term is third order in that error and
// is dropped: up to about 1e-12 |A| in the first step, which can still turn
// a chain's nearly degenerate pairs by more than 1e-5; the second step's
// closeness test (1/c = 1e-5) hands such pairs to its own Rayleigh-Ritz, and
// there the term is far below rounding.
// This replaces the published cluster threshold (a Frobenius-norm bound that
// is far too coarse for an FP32 starting point and lets badly conditioned
// Newton updates through) by a direct bound on the size of each update.
//
// Kernels per step: Y = A X, {S, G} = X^T {Y, X} and X M are dense FP64
// contractions on the matrix cores (v_mfma_f64_16x16x4f64): for batches of
// 193..208-row items whole-item products (one persistent work-group per CU;
// S and G stored as upper triangles, and the S, G product also forms the
// Rayleigh quotients and the close pairs), otherwise one work-group per
// 64 x 64 output tile of one item (S and G: upper tiles, mirrored) and
// refine_reach_kernel for the Rayleigh quotients and close pairs.  Readers
// of S and G take the upper triangle only.  form_m_kernel writes M = I + E
// outside the chains, refine_chain_kernel (one work-group per item) finds
// the chains and their Rayleigh-Ritz rotations.  A final kernel sorts the
// eigenpairs by eigenvalue and writes them to the caller's arrays.
#include <float.h>

#include "devutil.h"
#include "internal.h"

#include <type_traits>

namespace wpcd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;    // 4 wavefronts (per-item kernels, 64 x 64 GEMM tiles)
constexpr int kTM = 64;        // edge of the per-item kernels' GEMM tiles
constexpr int kTK = 32;        // reduction chunk
constexpr int kTileLds = kTK * kTM;  // doubles of one staged 64-row operand tile
// GEMM tile shapes: WR x WR wavefronts, each computing 32 x 32 (2 x 2 MFMA
// blocks of 16 x 16); the tile is 32 WR square, staged operands 32 WR x kTK.
template <int WR_>
struct TileCfg {
  static constexpr int WR = WR_;
  static constexpr int TM = 32 * WR_;          // tile edge
  static constexpr int NT = 64 * WR_ * WR_;    // threads
  static constexpr int LDS = kTK * TM;         // doubles of one staged operand
  static constexpr int HQ = (kTK / 4) * TM / NT;  // k quads staged per thread and operand
};
using T64 = TileCfg<2>;    // all products: 4 wavefronts, 64 x 64 tiles
// (128 x 128 tiles of 16 wavefronts halve the L2 reads per flop but ran
// slower: one such work-group fills a CU and its barriers stall all of it)
constexpr int kXcd = 8;        // XCDs; workgroups are dispatched to them round-robin
constexpr int kMaxChain = 64;  // columns of one LDS Rayleigh-Ritz batch
constexpr int kMaxBig = 24;    // longer chains per item, solved in device memory
constexpr int kBigRows = 19;   // rows per lane of their Jacobi (64 * 19 >= kMaxN)
// Closeness constant of refinement step st: c = 10^(close_log10 + 2 st) (by
// default 1e3 in the first step, which starts from FP32 vectors and admits
// Newton updates up to 1e-3; the second step, 1e5, admits updates up to 1e-5,
// whose second-order remainders stay near 1e-10 even for items whose FP32
// vectors were poor, and solves the larger residual rotations -- the first
// step's Newton remainders and the error of its chain blocks -- by
// Rayleigh-Ritz).

// One-dimensional grid of (item, tile) pairs in which every tile of an item
// lands on the same XCD (block b runs on XCD b mod 8), so that the item's
// operand panels are fetched into one L2 and re-read there by its other
// tiles.  The grid holds tiles * round_up(n_items, 8) blocks.
__device__ __forceinline__ bool xcd_item_tile(int tiles, int n_items, int& item, int& tile) {
  const int b = blockIdx.x;
  const int s = b / kXcd;
  item = (s / tiles) * kXcd + b % kXcd;
  tile = s % tiles;
  return item < n_items;
}
inline unsigned xcd_grid(int tiles, int n_items) {
  return (unsigned)tiles * (unsigned)((n_items + kXcd - 1) / kXcd * kXcd);
}

// --------------------------------------------------------------- GEMM tiles
// acc = sum_k A(m0+i, k) B(k, c0+j) over one 64 x 64 tile; A and B are
// operand views (below) giving A(i, k) and B(k, j) as op(i, k) / op(j, k).
// Operands are zero outside rows/cols/K.  The next 32-deep chunk is loaded
// into registers while the current one is multiplied; the loaded values are
// not touched until they are staged, so the loads stay in flight across the
// MFMAs of the current chunk.
// v_mfma_f64_16x16x4f64: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// D[i][j] in lane j + 16*(i % 4), register i / 4.
// Staging: thread t loads i = t % 64 and four consecutive k of one operand
// chunk (64 lanes along i per load: coalesced for sources contiguous in i,
// 32-byte row segments otherwise).  LDS layout: element (i, k) at
// T[k * 64 + (i ^ 16 (k & 1))].  A 64-bit LDS access is served per half
// wavefront (32 lanes over 64 four-byte banks): the stores (fixed k, 64 lanes
// over i) and the MFMA operand reads (16 lanes over i at k and at k + 1 in
// one half-wave, moved to opposite 16-double halves by the swizzle) then
// touch every bank once.

// ------------------------------------------------------------ operand views
// Dense matrix in device memory, element (i, k) at p[i * si + k * sk], read
// with raw buffer loads: an offset at or beyond the buffer's byte size reads
// zero, which pads rows >= n_i and k >= n_k without masking the data.
constexpr unsigned kOob = 0x40000000u;  // beyond every operand (< 12 MB each), no 32-bit wrap when added twice
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Mat {
  using raw_t = typename std::conditional<sizeof(T) == 8, u32x2, unsigned>::type;
  __amdgpu_buffer_rsrc_t r;
  int si, sk;
  __device__ Mat(const T* p, int64_t elems, int si_, int sk_) : si(si_), sk(sk_) {
    // word 3 = 0x00020000: raw (untyped) buffer access on gfx9 targets
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)(elems * (int64_t)sizeof(T)),
                                          0x00020000);
  }
  __device__ raw_t load(unsigned voff) const {
    if constexpr (sizeof(T) == 8)
      return __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
    else
      return __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0);
  }
  __device__ static double cvt(raw_t x) { return (double)__builtin_bit_cast(T, x); }
};
// A operand M^T or B operand M of an n x n row-major M (op(i, k) = M[k][i]: contiguous in i)
template <typename T>
__device__ Mat<T> col_view(const T* M, int rows_k, int ld) { return Mat<T>(M, (int64_t)rows_k * ld, 1, ld); }
// A operand M or B operand M^T (op(i, k) = M[i][k]: contiguous in k)
template <typename T>
__device__ Mat<T> row_view(const T* M, int rows_i, int ld) { return Mat<T>(M, (int64_t)rows_i * ld, ld, 1); }

template <class TC, typename T>
__device__ __forceinline__ void fetch(typename Mat<T>::raw_t (&r)[4 * TC::HQ], const Mat<T>& op, int r0, int k0,
                                      int n_i, int n_k) {
  const int tid = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(tid / TC::TM);  // wave-uniform
  const int i = r0 + tid % TC::TM;
  const unsigned base = i < n_i ? (unsigned)(i * op.si) * (unsigned)sizeof(T) : kOob;
#pragma unroll
  for (int h = 0; h < TC::HQ; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * (grp + (TC::NT / TC::TM) * h) + j;  // wave-uniform
      const unsigned ko = k < n_k ? (unsigned)(k * op.sk) * (unsigned)sizeof(T) : kOob;
      r[4 * h + j] = op.load(base + ko);
    }
}
template <class TC, class Op>
__device__ __forceinline__ void stash(double* T, const typename Op::raw_t (&r)[4 * TC::HQ]) {
  const int tid = threadIdx.x;
  const int i = tid % TC::TM, grp = tid / TC::TM;
#pragma unroll
  for (int h = 0; h < TC::HQ; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (grp + (TC::NT / TC::TM) * h) + j;
      T[k * TC::TM + (i ^ ((k & 1) << 4))] = Op::cvt(r[4 * h + j]);
    }
}

// The K loop for a wave whose live 16 x 16 sub-blocks are bi < NI, bj < NJ
// (NI = NJ = 0: the wave only helps staging).  NB = 1 or 2 B operands share
// the A operand (Bs holds NB staged tiles).
template <class TC, int NI, int NJ, int NB, class OA, class OB0, class OB1>
__device__ __forceinline__ void gemm_loop(double* As, double* Bs, int m0, int c0, int rows, int cols, int K,
                                          const OA& oa, const OB0& ob0, const OB1& ob1, d4 (&acc)[NB][2][2]) {
  constexpr int R = TC::TM;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = (wave / TC::WR) * 32, wc = (wave % TC::WR) * 32;
  typename OA::raw_t ra[4 * TC::HQ];
  typename OB0::raw_t rb0[4 * TC::HQ];
  typename OB1::raw_t rb1[4 * TC::HQ];
  fetch<TC>(ra, oa, m0, 0, rows, K);
  fetch<TC>(rb0, ob0, c0, 0, cols, K);
  if constexpr (NB > 1) fetch<TC>(rb1, ob1, c0, 0, cols, K);
  // this lane's read offsets for sub-block 0 / 1 at k = 4q + lane / 16: the
  // swizzle only depends on k & 1 = (lane / 16) & 1
  const int kk = lane >> 4, sw = (kk & 1) << 4;
  const int pa[2] = {kk * R + ((wr + (lane & 15)) ^ sw), kk * R + ((wr + 16 + (lane & 15)) ^ sw)};
  const int pb[2] = {kk * R + ((wc + (lane & 15)) ^ sw), kk * R + ((wc + 16 + (lane & 15)) ^ sw)};
  auto quad = [&](int q) {
    const int o = q * 4 * R;
    double a[2], b[NB][2];
#pragma unroll
    for (int bi = 0; bi < NI; ++bi) a[bi] = As[o + pa[bi]];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int bj = 0; bj < NJ; ++bj) b[nb][bj] = Bs[nb * TC::LDS + o + pb[bj]];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int bi = 0; bi < NI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NJ; ++bj)
          acc[nb][bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[nb][bj], acc[nb][bi][bj], 0, 0, 0);
  };
  for (int k0 = 0; k0 < K; k0 += kTK) {
    __syncthreads();  // previous chunk fully consumed
    stash<TC, OA>(As, ra);
    stash<TC, OB0>(Bs, rb0);
    if constexpr (NB > 1) stash<TC, OB1>(Bs + TC::LDS, rb1);
    __syncthreads();
    if (k0 + kTK < K) {
      fetch<TC>(ra, oa, m0, k0 + kTK, rows, K);
      fetch<TC>(rb0, ob0, c0, k0 + kTK, cols, K);
      if constexpr (NB > 1) fetch<TC>(rb1, ob1, c0, k0 + kTK, cols, K);
    }
    if constexpr (NI > 0 && NJ > 0) {
      if (K - k0 >= kTK) {
        if constexpr (NB == 1) {
#pragma unroll
          for (int q = 0; q < kTK / 4; ++q) quad(q);
        } else {  // two accumulator sets: keep fewer quads in flight (registers)
#pragma unroll 2
          for (int q = 0; q < kTK / 4; ++q) quad(q);
        }
      } else {
        const int qend = (K - k0 + 3) >> 2;
        for (int q = 0; q < qend; ++q) quad(q);
      }
    }
  }
}

template <class TC, int NB, class OA, class OB0, class OB1>
__device__ void gemm_core(double* As, double* Bs, int m0, int c0, int rows, int cols, int K, const OA& oa,
                          const OB0& ob0, const OB1& ob1, d4 (&acc)[NB][2][2]) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = (wave / TC::WR) * 32, wc = (wave % TC::WR) * 32;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[nb][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  const int ni = (m0 + wr < rows) + (m0 + wr + 16 < rows);
  const int nj = (c0 + wc < cols) + (c0 + wc + 16 < cols);
  if (ni == 2 && nj == 2)
    gemm_loop<TC, 2, 2, NB>(As, Bs, m0, c0, rows, cols, K, oa, ob0, ob1, acc);
  else if (ni == 2 && nj == 1)
    gemm_loop<TC, 2, 1, NB>(As, Bs, m0, c0, rows, cols, K, oa, ob0, ob1, acc);
  else if (ni == 1 && nj == 2)
    gemm_loop<TC, 1, 2, NB>(As, Bs, m0, c0, rows, cols, K, oa, ob0, ob1, acc);
  else if (ni == 1 && nj == 1)
    gemm_loop<TC, 1, 1, NB>(As, Bs, m0, c0, rows, cols, K, oa, ob0, ob1, acc);
  else
    gemm_loop<TC, 0, 0, NB>(As, Bs, m0, c0, rows, cols, K, oa, ob0, ob1, acc);
}

template <class TC, class OA, class OB>
__device__ __forceinline__ void gemm_tile(double* As, double* Bs, int m0, int c0, int rows, int cols, int K,
                                          const OA& oa, const OB& ob, d4 (&acc)[2][2]) {
  gemm_core<TC, 1>(As, Bs, m0, c0, rows, cols, K, oa, ob, ob, reinterpret_cast<d4(&)[1][2][2]>(acc));
}

template <class TC, class G>
__device__ __forceinline__ void tile_store(int m0, int c0, int rows, int cols, const d4 (&acc)[2][2], const G& g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / TC::WR) * 32, wc = (wave % TC::WR) * 32;
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

// Newton correction E(k,j) from g = G_kj, s = S_kj and the Rayleigh quotients
// lk, lj: for k != j the first-order update (R_kj/2 for a close pair), R_jj/2
// on the diagonal
__device__ __forceinline__ double newton_e_of(double g, double s, double lk, double lj, bool diag, double closec) {
  if (diag) return 0.5 * (1.0 - g);
  const double r = -g;
  const double d = fabs(lj - lk);
  const double num = s + lj * r;
  if (closec * fabs(num) >= d || closec * fabs(s + lk * r) >= d) return 0.5 * r;
  return num / (lj - lk);
}
__device__ __forceinline__ int64_t upper_at(int n, int k, int j) {
  return k <= j ? (int64_t)k * n + j : (int64_t)j * n + k;
}
__device__ __forceinline__ double newton_e(const double* S, const double* G, const double* lam, int n, int k,
                                           int j, double closec) {
  const int64_t e = upper_at(n, k, j);
  return newton_e_of(G[e], S[e], lam[k], lam[j], j == k, closec);
}

// Per-item work-space (doubles): P1 | Y | S | G | W5 | W6 | W7, each n*n.
struct WS {
  double *P1, *Y, *S, *G, *W5, *W6, *W7;
  __device__ WS(double* work, const ItemDev& it) {
    const int64_t nn = (int64_t)it.n * it.n;
    P1 = work + it.w_off;
    Y = P1 + nn;
    S = Y + nn;
    G = S + nn;
    W5 = G + nn;
    W6 = W5 + nn;
    W7 = W6 + nn;
  }
};

// ------------------------------------------------------------ step kernels
// One-dimensional grids over (item, tile) from xcd_item_tile.
#define WPCD_LDS_TILES(TC, NB)    \
  __shared__ double As[TC::LDS]; \
  __shared__ double Bs[(NB) * TC::LDS]

// Y = H X = V X + H0 X (H0 diagonal)
template <typename XT>
__global__ __launch_bounds__(T64::NT, 3) void gemm_y_kernel(const ItemDev* __restrict__ items, int n_items,
                                                        const GridDev* __restrict__ grids,
                                                        const double* __restrict__ v64, const XT* xin, int xin_ws,
                                                        double* work, int tiles) {
  WPCD_LDS_TILES(T64, 1);
  int item, tile;
  if (!xcd_item_tile(tiles, n_items, item, tile)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nt = (n + T64::TM - 1) / T64::TM;
  if (tile >= nt * nt) return;
  const int tm = tile / nt, tc = tile % nt;
  const GridDev g = grids[it.grid];
  const WS ws(work, it);
  const XT* X = xin_ws ? reinterpret_cast<const XT*>(ws.P1) : (xin + it.v_off);
  d4 acc[2][2];
  // V is symmetric: its rows are read as columns (contiguous along the tile's rows)
  gemm_tile<T64>(As, Bs, tm * T64::TM, tc * T64::TM, n, n, n, col_view(v64 + it.v_off, n, n), col_view(X, n, n), acc);
  double* Y = ws.Y;
  const int N = it.N;
  tile_store<T64>(tm * T64::TM, tc * T64::TM, n, n, acc, [&](int r, int c, double v) {
    Y[(int64_t)r * n + c] = fma(g.e0[r % N], (double)X[(int64_t)r * n + c], v);  // + H0 X
  });
}

// S = X^T Y and G = X^T X in one pass over the shared operand X^T, on the
// upper tiles (tm <= tc), mirrored on store
template <typename XT>
__global__ __launch_bounds__(T64::NT) void gemm_sg_kernel(const ItemDev* __restrict__ items, int n_items,
                                                        const XT* xin, int xin_ws, double* work, int tiles) {
  WPCD_LDS_TILES(T64, 2);
  int item, t;
  if (!xcd_item_tile(tiles, n_items, item, t)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nt = (n + T64::TM - 1) / T64::TM;
  int tm = 0;
  while (tm < nt && t >= nt - tm) {
    t -= nt - tm;
    ++tm;
  }
  if (tm >= nt) return;
  const int tc = tm + t;
  const WS ws(work, it);
  const XT* X = xin_ws ? reinterpret_cast<const XT*>(ws.P1) : (xin + it.v_off);
  d4 acc[2][2][2];
  gemm_core<T64, 2>(As, Bs, tm * T64::TM, tc * T64::TM, n, n, n, col_view(X, n, n), col_view<double>(ws.Y, n, n),
                    col_view(X, n, n), acc);
  double* S = ws.S;
  double* G = ws.G;
  tile_store<T64>(tm * T64::TM, tc * T64::TM, n, n, acc[0], [&](int r, int c, double v) {
    if (r > c) return;  // one writer per symmetric pair
    S[(int64_t)r * n + c] = v;
    S[(int64_t)c * n + r] = v;
  });
  tile_store<T64>(tm * T64::TM, tc * T64::TM, n, n, acc[1], [&](int r, int c, double v) {
    if (r > c) return;
    G[(int64_t)r * n + c] = v;
    G[(int64_t)c * n + r] = v;
  });
}

// Columns of M = I + E outside chains, row-major into W6 (the chain kernel
// writes the chain columns, possibly at the same time on another stream).
// Exclusive scan of one int per thread over the work-group (thread order),
// by addition or by maximum (identity -1: the values scanned by maximum are
// column indices); total receives the whole group's result.  Every thread
// of the work-group must call it; sh holds kBlock/64 ints.  Ends with a
// barrier, so sh can be reused at once.
template <bool MAX>
__device__ int block_xscan(int v, int* sh, int& total) {
  constexpr int kIdent = MAX ? -1 : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x = MAX ? max(x, y) : x + y;
  }
  if (lane == 63) sh[wave] = x;
  int ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = kIdent;
  __syncthreads();
  int pre = kIdent, tot = kIdent;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wave) pre = MAX ? max(pre, sh[w]) : pre + sh[w];
    tot = MAX ? max(tot, sh[w]) : tot + sh[w];
  }
  __syncthreads();
  total = tot;
  return MAX ? max(pre, ex) : pre + ex;
}

// cl holds reach[p] from refine_reach_kernel: column j lies in a chain iff
// some interval [p, reach[p]] with reach[p] > p covers it, i.e. reach[j] > j
// or max_{p<j} reach[p] >= j (a prefix maximum over the work-group).  lam_pre
// holds the Rayleigh quotients E was built from.  S and G are read from their
// upper triangles only (the whole-item S, G product stores nothing else): one
// work-group per (item, pair of 32-row blocks I <= J) from xcd_item_tile
// reads the upper tile (I, J) once and writes both M[k][j] (k in I, j in J,
// k <= j) and M[j][k] (k < j, from the same S_kj and G_kj) through a
// transposed copy in LDS, so every store covers consecutive columns.
constexpr int kFT = 32;                    // form_m tile edge
constexpr int kFRY = kBlock / kFT;         // tile rows per round
constexpr int kFRows = kFT / kFRY;         // rounds (loads issued before use)
inline int form_m_tiles(int max_n) {
  const int nb = (max_n + kFT - 1) / kFT;
  return nb * (nb + 1) / 2;
}
__global__ __launch_bounds__(kBlock) void form_m_kernel(const ItemDev* __restrict__ items,
                                                        const double* __restrict__ lam_pre, double* work,
                                                        const int32_t* __restrict__ cl, double closec, int tiles,
                                                        int n_items) {
  __shared__ double tt[kFT * (kFT + 1)];
  __shared__ double lam_i[kFT], lam_j[kFT];
  __shared__ unsigned char in_i[kFT], in_j[kFT];
  __shared__ int scan_sh[kBlock / 64];
  int item, tile;
  if (!xcd_item_tile(tiles, n_items, item, tile)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nb = (n + kFT - 1) / kFT;
  if (tile >= nb * (nb + 1) / 2) return;
  int bi = 0, rem = tile;  // tile -> (I, J), row by row over the upper block triangle
  while (rem >= nb - bi) {
    rem -= nb - bi;
    ++bi;
  }
  const int i0 = bi * kFT, j0 = (bi + rem) * kFT;
  const WS ws(work, it);
  // the tile's S and G loads go out first: they do not wait for the chain scan
  const int tx = threadIdx.x & (kFT - 1), ty = threadIdx.x / kFT;
  const int j = j0 + tx;
  double gv[kFRows], sv[kFRows];
#pragma unroll
  for (int u = 0; u < kFRows; ++u) {
    const int k = i0 + ty + kFRY * u;
    const int64_t e = (k < n && j < n && k <= j) ? (int64_t)k * n + j : 0;
    gv[u] = ws.G[e];
    sv[u] = ws.S[e];
  }
  {
    // chain membership of the tile's rows and columns (no reach list: no chains)
    const int per = (n + kBlock - 1) / kBlock;
    const int a0 = min(n, (int)threadIdx.x * per), a1 = min(n, a0 + per);
    int lm = -1;
    for (int c = a0; c < a1; ++c) lm = max(lm, cl ? cl[it.e_off + c] : c);
    int tot;
    int cover = block_xscan<true>(lm, scan_sh, tot);
    for (int c = a0; c < a1; ++c) {
      const int rc = cl ? cl[it.e_off + c] : c;
      const unsigned char v = (rc > c || cover >= c) ? 1 : 0;
      if (c >= i0 && c < i0 + kFT) in_i[c - i0] = v;
      if (c >= j0 && c < j0 + kFT) in_j[c - j0] = v;
      cover = max(cover, rc);
    }
    if (threadIdx.x < kFT) {
      const int t = threadIdx.x;
      lam_i[t] = i0 + t < n ? lam_pre[it.e_off + i0 + t] : 0.0;
      lam_j[t] = j0 + t < n ? lam_pre[it.e_off + j0 + t] : 0.0;
    }
  }
  __syncthreads();
  if (j < n) {
    const double lj = lam_j[tx];
#pragma unroll
    for (int u = 0; u < kFRows; ++u) {
      const int kk = ty + kFRY * u, k = i0 + kk;
      if (k >= n || k > j) continue;
      const double lk = lam_i[kk];
      if (!in_j[tx]) ws.W6[(int64_t)k * n + j] = (k == j ? 1.0 : 0.0) + newton_e_of(gv[u], sv[u], lk, lj, k == j, closec);
      if (k < j) tt[tx * (kFT + 1) + kk] = newton_e_of(gv[u], sv[u], lj, lk, false, closec);
    }
  }
  __syncthreads();
  // M[j][k] for the tile's columns j (rows of M) and rows k (columns of M)
#pragma unroll
  for (int u = 0; u < kFRows; ++u) {
    const int jj = ty + kFRY * u, jr = j0 + jj, k = i0 + tx;
    if (jr < n && k < jr && !in_i[tx]) ws.W6[(int64_t)jr * n + k] = tt[jj * (kFT + 1) + tx];
  }
}

// X' = X M with M in W6 (form_m_kernel and refine_chain_kernel).
template <typename XT>
__global__ __launch_bounds__(T64::NT, 3) void gemm_xm_kernel(const ItemDev* __restrict__ items, int n_items,
                                                         const XT* xin, int xin_ws, double* evec, int xout_ws,
                                                         double* work, int tiles) {
  WPCD_LDS_TILES(T64, 1);
  int item, tile;
  if (!xcd_item_tile(tiles, n_items, item, tile)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nt = (n + T64::TM - 1) / T64::TM;
  if (tile >= nt * nt) return;
  const int tm = tile / nt, tc = tile % nt;
  const WS ws(work, it);
  const XT* X = xin_ws ? reinterpret_cast<const XT*>(ws.P1) : (xin + it.v_off);
  double* Xo = xout_ws ? ws.P1 : (evec + it.v_off);
  d4 acc[2][2];
  gemm_tile<T64>(As, Bs, tm * T64::TM, tc * T64::TM, n, n, n, row_view(X, n, n), col_view<double>(ws.W6, n, n), acc);
  tile_store<T64>(tm * T64::TM, tc * T64::TM, n, n, acc, [&](int r, int c, double v) { Xo[(int64_t)r * n + c] = v; });
}

// ------------------------------------------------------------ reach kernel
// Rayleigh quotients lam_i = S_ii/G_ii (-> lam_pre) and, per row p, the
// largest q > p with (p, q) close (else p; -> cl, read back by the chain
// kernel).  One-dimensional grid over (item, block of kReachRows rows) from
// xcd_item_tile, so the blocks of an item share one L2 for the diagonal
// reads; 8 wavefronts, each taking kReachRPW rows (p = block row + wave + 8 r)
// with lanes over q (coalesced reads of rows of S and G); the loads of all
// its rows for kReachChunks chunks of 64 columns are issued before any is
// tested (S and G come from HBM).
constexpr int kReachWaves = 8;
constexpr int kReachRPW = 4;
constexpr int kReachRows = kReachWaves * kReachRPW;
constexpr int kReachChunks = 4;
__global__ __launch_bounds__(64 * kReachWaves) void refine_reach_kernel(const ItemDev* __restrict__ items,
                                                                        double* __restrict__ lam_pre,
                                                                        const double* work, int32_t* __restrict__ cl,
                                                                        double closec, int tiles, int n_items) {
  __shared__ double lam[kMaxN];
  int item, tile;
  if (!xcd_item_tile(tiles, n_items, item, tile)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  if (tile * kReachRows >= n) return;
  const WS ws(const_cast<double*>(work), it);
  const double* S = ws.S;
  const double* G = ws.G;
  for (int i = threadIdx.x; i < n; i += 64 * kReachWaves) lam[i] = S[(int64_t)i * n + i] / G[(int64_t)i * n + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p0 = tile * kReachRows + w;
  int rq[kReachRPW];
#pragma unroll
  for (int r = 0; r < kReachRPW; ++r) rq[r] = p0 + kReachWaves * r;
  // chunk c of row p covers q = p + 1 + 64 c + lane
  const int nchunk = (n - p0 - 1 + 63) / 64;  // of the wave's first (longest) row
  for (int c0 = 0; c0 < nchunk; c0 += kReachChunks) {
    double sv[kReachRPW][kReachChunks], gv[kReachRPW][kReachChunks];
#pragma unroll
    for (int r = 0; r < kReachRPW; ++r)
#pragma unroll
      for (int c = 0; c < kReachChunks; ++c) {
        const int p = p0 + kReachWaves * r, q = p + 1 + 64 * (c0 + c) + lane;
        const int64_t e = (p < n && q < n) ? (int64_t)p * n + q : 0;
        sv[r][c] = S[e];
        gv[r][c] = G[e];
      }
#pragma unroll
    for (int r = 0; r < kReachRPW; ++r) {
      const int p = p0 + kReachWaves * r;
      if (p >= n) continue;
      const double lp = lam[p];
#pragma unroll
      for (int c = 0; c < kReachChunks; ++c) {
        const int q = p + 1 + 64 * (c0 + c) + lane;
        if (q >= n) continue;
        const double rr = -gv[r][c];
        const double d = fabs(lam[q] - lp);
        if (closec * fabs(sv[r][c] + lam[q] * rr) >= d || closec * fabs(sv[r][c] + lp * rr) >= d) rq[r] = q;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kReachRPW; ++r) {
    int v = rq[r];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    const int p = p0 + kReachWaves * r;
    if (lane == 0 && p < n) {
      cl[it.e_off + p] = v;
      lam_pre[it.e_off + p] = lam[p];
    }
  }
}

// One-sided Jacobi on the chains of a Rayleigh-Ritz batch: column j of W
// (leading dimension ldw) holds only the rows of its own chain, at offsets
// 0 .. len - 1 from the chain's first column, and zeros up to G * RMAX (the
// off-chain entries of the block-diagonal matrix are not stored).  The
// chains are independent, so each runs its own round-robin ordering over
// its own rows, and all chains advance together -- a sweep has
// max(ne_c) - 1 barrier-separated steps instead of Tb - 1.  bstart/blen: the
// batch's chains (batch-local first column, length), nb of them; poff[c] =
// sum of (len+1)/2 over earlier chains; pch[i]: the chain of the batch's pair
// slot i (poff[c] <= i < poff[c + 1]).  Column loads and stores need no
// guard (rotations keep the zero rows zero), and the squared column norms
// (nrm, Tb doubles of LDS) are tracked through the rotations from exact
// values at the start of every sweep: one dot product per pair.  Same skip
// test (cosine above tol), stopping rule (a sweep whose largest rotated
// cosine is below stop) and return value as onesided_jacobi_lds.
template <int BLOCK, int G, int RMAX>
__device__ __forceinline__ int chain_jacobi(double* W, int ldw, int Tb, const short* bstart, const short* blen,
                                            const short* poff, const unsigned char* pch, int nb, double* nrm,
                                            double tol, double stop, int max_sweeps, int* rot_flag) {
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  constexpr int ngrp = BLOCK / G;
  int ne_max = 0;
  for (int c = 0; c < nb; ++c) ne_max = max(ne_max, (blen[c] + 1) & ~1);
  const int ptot = poff[nb];
  // this group's pair slots (idx = grp + s ngrp): chain, length, first
  // column and round-robin positions, fixed for the whole iteration; the
  // positions advance by one per step (rr_index without its division)
  constexpr int kSlots = 2;
  static_assert(kSlots * ngrp >= kMaxChain / 2 + kMaxChain / 4, "pair slots of a batch");
  int sm[kSlots], sne[kSlots], sb0[kSlots], sp0[kSlots], sq0[kSlots];
#pragma unroll
  for (int sl = 0; sl < kSlots; ++sl) {
    const int idx = grp + sl * ngrp;
    sm[sl] = 0;
    if (idx < ptot) {
      const int c = pch[idx];
      sm[sl] = blen[c];
      sne[sl] = (sm[sl] + 1) & ~1;
      sb0[sl] = bstart[c];
      const int pr = idx - poff[c];
      sp0[sl] = pr;                 // position of the first index
      sq0[sl] = sne[sl] - 1 - pr;   // position of the second
    }
  }
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int j = grp; j < Tb; j += ngrp) {
      const double* c = W + j * ldw + lane;
      double s2 = 0.0;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) s2 = fma(c[k * G], c[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm[j] = s2;
    }
    __syncthreads();
    float cmax = 0.0f;  // largest rotated cosine of this lane's pairs in the sweep
    // (pos - 1 + step) mod (ne - 1) of each slot's two positions
    int vp[kSlots], vq[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      vp[sl] = sp0[sl] - 1;
      vq[sl] = sq0[sl] - 1;
    }
    for (int step = 0; step < ne_max - 1; ++step) {
#pragma unroll
      for (int sl = 0; sl < kSlots; ++sl) {
        const int m = sm[sl], ne = sne[sl], b0 = sb0[sl];
        if (m == 0 || step >= ne - 1) continue;
        const int p = sp0[sl] == 0 ? 0 : 1 + vp[sl];
        const int q = sq0[sl] == 0 ? 0 : 1 + vq[sl];
        if (++vp[sl] == ne - 1) vp[sl] = 0;
        if (++vq[sl] == ne - 1) vq[sl] = 0;
        if (p >= m || q >= m) continue;
        double* wp = W + (b0 + p) * ldw + lane;
        double* wq = W + (b0 + q) * ldw + lane;
        double xp[RMAX], xq[RMAX];
        double ga = 0.0;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
          xp[k] = wp[k * G];
          xq[k] = wq[k * G];
          ga = fma(xp[k], xq[k], ga);
        }
        ga = group_sum<G>(ga);
        const double al = nrm[b0 + p], be = nrm[b0 + q];
        // cosine |w_p.w_q| / (|w_p||w_q|) (a zero column gives NaN: no rotation)
        const double cosv = fabs(ga) * rsqrt(al * be);
        if (cosv > tol) {
          // the rotation of hestenes_rotation written with one division:
          // with d = be - al, g = 2 ga, zeta = d/g and
          // t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)) = sign(d) g/(|d| + sqrt(d^2 + g^2))
          const double d = be - al, g = 2.0 * ga;
          const double t = copysign(1.0, d) * g / (fabs(d) + sqrt(fma(d, d, g * g)));
          const double cs = rsqrt(fma(t, t, 1.0)), sn = cs * t;
#pragma unroll
          for (int k = 0; k < RMAX; ++k) {
            wp[k * G] = cs * xp[k] - sn * xq[k];
            wq[k * G] = sn * xp[k] + cs * xq[k];
          }
          if (lane == 0) {
            nrm[b0 + p] = al - t * ga;
            nrm[b0 + q] = be + t * ga;
          }
          cmax = fmaxf(cmax, (float)cosv);
        }
      }
      __syncthreads();
    }
    // the sweep's largest rotation: wavefront maximum, one LDS atomic per wavefront
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) cmax = fmaxf(cmax, __shfl_xor(cmax, off, 64));
    if ((threadIdx.x & 63) == 0 && cmax > 0.0f) atomicMax(&rot_flag[sweep], __float_as_int(cmax));
    __syncthreads();
    if (__int_as_float(rot_flag[sweep]) < (float)stop) return sweep + 1;
  }
  return max_sweeps + 1;
}

// Chains of one item from its reach list in LDS: the unions of overlapping
// [p, reach[p]] (reach[p] >= p) with at least two columns.  Column i opens a
// new segment iff every reach[p] with p < i is below i, so the segments
// follow from a prefix maximum of reach, and each chain's position among all
// chain columns from prefix sums over the segments (all chains of up to
// kMaxChain columns first, then the long ones of the list).  reach is
// overwritten in place with each column's chain position (>= 0), -1 (single
// column) or -2 (a long chain beyond the list of kMaxBig: its columns get
// I + E and the item is flagged).  Chains of up to kMaxChain columns go to
// ch_start/ch_len (*s_nch of them), long ones to big_start/big_len
// (*s_nbig); *s_fail is set when the list overflows.  Every thread of the
// work-group calls it; it ends with a barrier.
__device__ void find_chains(int n, int* reach, short* seg_start, int* scan_sh, short* ch_start, short* ch_len,
                            short* big_start, short* big_len, int* s_nch, int* s_nbig, int* s_fail) {
  {
    const int per = (n + kBlock - 1) / kBlock;
    const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
    int lm = -1;
    for (int i = i0; i < i1; ++i) lm = max(lm, reach[i]);
    int tot;
    const int pm0 = block_xscan<true>(lm, scan_sh, tot);
    int pm = pm0, ns = 0;
    for (int i = i0; i < i1; ++i) {
      ns += pm < i ? 1 : 0;
      pm = max(pm, reach[i]);
    }
    int nseg;
    int sid = block_xscan<false>(ns, scan_sh, nseg);
    pm = pm0;
    for (int i = i0; i < i1; ++i) {
      if (pm < i) seg_start[sid++] = (short)i;
      pm = max(pm, reach[i]);
    }
    __syncthreads();
    // per segment: (chain count << 16 | chain columns), (long count << 16 | long columns)
    const int sper = (nseg + kBlock - 1) / kBlock;
    const int s0 = min(nseg, (int)threadIdx.x * sper), s1 = min(nseg, s0 + sper);
    int vc = 0, vb = 0;
    for (int g = s0; g < s1; ++g) {
      const int m = (g + 1 < nseg ? seg_start[g + 1] : n) - seg_start[g];
      if (m >= 2 && m <= kMaxChain) vc += (1 << 16) + m;
      if (m > kMaxChain) vb += (1 << 16) + m;
    }
    int tc, tb;
    int xc = block_xscan<false>(vc, scan_sh, tc);
    int xb = block_xscan<false>(vb, scan_sh, tb);
    const int tcols = tc & 0xffff;
    for (int g = s0; g < s1; ++g) {
      const int i = seg_start[g], m = (g + 1 < nseg ? seg_start[g + 1] : n) - i;
      if (m >= 2 && m <= kMaxChain) {
        const int c = xc >> 16, T0 = xc & 0xffff;
        ch_start[c] = (short)i;
        ch_len[c] = (short)m;
        for (int t = 0; t < m; ++t) reach[i + t] = T0 + t;
        xc += (1 << 16) + m;
      } else if (m > kMaxChain) {
        const int b = xb >> 16, T0 = tcols + (xb & 0xffff);
        if (b < kMaxBig) {
          big_start[b] = (short)i;
          big_len[b] = (short)m;
        }
        for (int t = 0; t < m; ++t) reach[i + t] = b < kMaxBig ? T0 + t : -2;
        xb += (1 << 16) + m;
      } else {
        reach[i] = -1;
      }
    }
    if (threadIdx.x == 0) {
      *s_nch = tc >> 16;
      *s_nbig = min(tb >> 16, kMaxBig);
      *s_fail = (tb >> 16) > kMaxBig ? 1 : 0;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ chain kernel
// One work-group per item: Rayleigh quotients, close pairs and chains, and the
// Rayleigh-Ritz rotation of every chain.  Chains of up to kMaxChain columns
// are processed in batches of whole chains with at most kMaxChain columns;
// for a batch with columns cols[0..Tb): P -> W5 (n x Tb), T -> Y (n x Tb),
// P^T T -> LDS (only the diagonal blocks, one per chain, are kept), which
// gives P^T S P with the rows C of T and S, one-sided Jacobi, Q -> LDS, and
// P Q -> the batch's columns of M (n x n, W6).
// Longer chains (dense parts of the spectrum of large items) are left to
// refine_bigchain_kernel, their list at the end of the item's W7.  Writes the
// refined eigenvalues of its chains to eval, the Rayleigh quotients outside
// chains; the other columns of M come from form_m_kernel.
__global__ __launch_bounds__(kBlock, 2) void refine_chain_kernel(const ItemDev* __restrict__ items,
                                                              double* __restrict__ lam_pre,
                                                              double* __restrict__ eval, double* work,
                                                              int32_t* __restrict__ cl,
                                                              int32_t* __restrict__ status, double closec,
                                                              double jtol, double jstop) {
  // column stride of the chain matrix: 72 = 8 (mod 32) doubles, so the
  // columns read by the four 8-lane groups of a half wavefront in one step
  // (consecutive chain positions) start 16 banks apart and cover all 64 banks
  constexpr int ldw = 72;
  // the chain matrix W of a batch shares LDS with the GEMM staging tiles: it
  // is written after the P^T S P product's last chunk and read into Q before
  // the P Q product stages its first one
  constexpr int kSmem = (2 * kTileLds > kMaxChain * ldw) ? 2 * kTileLds : kMaxChain * ldw;
  __shared__ double smem[kSmem];
  double* const As = smem;
  double* const Bs = smem + kTileLds;
  double* const W = smem;
  __shared__ double lam[kMaxN];
  __shared__ int reach[kMaxN];
  __shared__ short ch_start[kMaxN / 2];
  __shared__ short ch_len[kMaxN / 2];
  __shared__ double shift[kMaxChain];
  __shared__ double nrm[kMaxChain];
  __shared__ int cols[kMaxChain];
  __shared__ int blk[kMaxChain];
  __shared__ int rot_flag[64];
  __shared__ short big_start[kMaxBig], big_len[kMaxBig];
  __shared__ short bt_start[kMaxChain / 2], bt_len[kMaxChain / 2], bt_poff[kMaxChain / 2 + 1];
  __shared__ short bend[kMaxChain];
  __shared__ short src[kMaxChain];
  __shared__ unsigned char pch[kMaxChain];
  __shared__ int s_nch, s_c0, s_c1, s_Tb, s_fail, s_nbig, s_nbt;
  __shared__ short seg_start[kMaxN];
  __shared__ int scan_sh[kBlock / 64];
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  const WS ws(work, it);
  const double* S = ws.S;
  const double* G = ws.G;
  // Rayleigh quotients and reach[p] from refine_reach_kernel (reach staged in cl)
  for (int i = threadIdx.x; i < n; i += kBlock) {
    lam[i] = lam_pre[it.e_off + i];
    reach[i] = cl[it.e_off + i];
  }
  __syncthreads();
  // the chain positions stay in LDS: cl is read-only here, because
  // form_m_kernel reads the same reach list from cl at the same time on the
  // side stream
  find_chains(n, reach, seg_start, scan_sh, ch_start, ch_len, big_start, big_len, &s_nch, &s_nbig, &s_fail);
  if (threadIdx.x == 0) s_c1 = 0;
  // the long chains go to refine_bigchain_kernel: their list at the end of
  // the item's W7 (the batches below use its first kMaxChain^2 doubles)
  if (threadIdx.x == 0 && n > kMaxChain) {
    double* tail = ws.W7 + (int64_t)n * n - (2 * kMaxBig + 1);
    tail[0] = (double)s_nbig;
    for (int b = 0; b < s_nbig; ++b) {
      tail[1 + 2 * b] = (double)big_start[b];
      tail[2 + 2 * b] = (double)big_len[b];
    }
  }
  // columns of chains beyond the list: M = I + E (form_m_kernel takes them
  // for chain columns)
  if (s_fail)
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kBlock) {
      const int k = (int)(e / n), j = (int)(e - (int64_t)k * n);
      if (reach[j] == -2) ws.W6[e] = (k == j ? 1.0 : 0.0) + newton_e(S, G, lam, n, k, j, closec);
    }
  const int nch = s_nch;
  const int nt = (n + kTM - 1) / kTM;
  double* P = ws.W5;   // n x Tb
  double* TS = ws.Y;   // n x Tb: T = S_C + Lam E / 2
  double* M = ws.W6;  // n x n update matrix (chain columns)
  double* QB = ws.W7;  // Tb x Tb sorted Q of a batch (W7 holds a long chain's matrix later)
  d4 acc[2][2];
  while (true) {
    // next batch: chains [c0, c1) with at most kMaxChain columns in total
    // (thread 0 picks them, then every thread fills the per-column tables)
    if (threadIdx.x == 0) {
      const int c0 = s_c1;
      int c1 = c0, Tb = 0, nbt = 0;
      bt_poff[0] = 0;
      while (c1 < nch && Tb + ch_len[c1] <= kMaxChain) {
        bt_start[nbt] = (short)Tb;
        bt_len[nbt] = ch_len[c1];
        bt_poff[nbt + 1] = (short)(bt_poff[nbt] + (ch_len[c1] + 1) / 2);
        ++nbt;
        Tb += ch_len[c1];
        ++c1;
      }
      s_c0 = c0;
      s_c1 = c1;
      s_Tb = Tb;
      s_nbt = nbt;
    }
    __syncthreads();
    const int Tb = s_Tb, c0 = s_c0;
    if (Tb == 0) break;
    if (threadIdx.x < kMaxChain) {
      const int nbt = s_nbt, t = threadIdx.x;
      int b = 0;  // the batch chain of column t, and of pair slot t
      while (b + 1 < nbt && bt_start[b + 1] <= t) ++b;
      if (t < Tb) {
        cols[t] = ch_start[c0 + b] + (t - bt_start[b]);
        blk[t] = bt_start[b];
        bend[t] = (short)(bt_start[b] + bt_len[b]);
      }
      int bp = 0;
      while (bp + 1 < nbt && bt_poff[bp + 1] <= t) ++bp;
      if (t < bt_poff[nbt]) pch[t] = (unsigned char)bp;
    }
    __syncthreads();
    // P and T: each wavefront splits into row groups of tpw >= Tb lanes (8,
    // 16, 32 or 64), lane t of a group takes column t; the groups of all
    // wavefronts interleave the rows (all loads of a round of 8 rows per
    // group are issued before their use: S and G come from HBM)
    const int tpw = Tb <= 8 ? 8 : Tb <= 16 ? 16 : Tb <= 32 ? 32 : 64;
    if ((int)(threadIdx.x & (tpw - 1)) < Tb) {
      const int t = threadIdx.x & (tpw - 1), j = cols[t];
      const double lj = lam[j];
      constexpr int U = 8, KS = kBlock / 64;
      const int gpw = 64 / tpw, RS = KS * gpw;  // groups per wavefront, row stride
      for (int k0 = (threadIdx.x >> 6) * gpw + ((threadIdx.x & 63) / tpw); k0 < n; k0 += U * RS) {
        double gv[U], sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = upper_at(n, min(k0 + u * RS, n - 1), j);
          gv[u] = G[e];
          sv[u] = S[e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * RS;
          if (k < n) {
            const double e = newton_e_of(gv[u], sv[u], lam[k], lj, k == j, closec);
            P[(int64_t)k * Tb + t] = (k == j ? 1.0 : 0.0) + e;
            TS[(int64_t)k * Tb + t] = fma(0.5 * lam[k], e, sv[u]);
          }
        }
      }
    }
    __syncthreads();
    // V = P^T T = T_C + E^T S_C + E^T Lam E / 2, then P^T S P ~ V + V^T - T_C - T_C^T + S_CC
    gemm_tile<T64>(As, Bs, 0, 0, Tb, Tb, n, col_view<double>(P, n, Tb), col_view<double>(TS, n, Tb), acc);
    __syncthreads();  // W overlays the staging tiles
    // each column holds its chain's rows from offset 0 (V as it is, made
    // symmetric below), zeros below them up to kMaxChain
    tile_store<T64>(0, 0, Tb, Tb, acc, [&](int r, int cc, double v) {
      if (blk[r] == blk[cc]) W[cc * ldw + (r - blk[cc])] = v;
    });
    for (int e = threadIdx.x; e < Tb * kMaxChain; e += kBlock) {
      const int j = e / kMaxChain, r = e - j * kMaxChain;
      if (r >= bend[j] - blk[j]) W[j * ldw + r] = 0.0;
    }
    if (threadIdx.x < 64) rot_flag[threadIdx.x] = 0;
    __syncthreads();
    // one thread per unordered same-chain pair (a <= b, batch positions);
    // the loads of two pairs are issued before either is used
    for (int e0 = threadIdx.x; e0 < Tb * kMaxChain; e0 += 2 * kBlock) {
      double tv[2][3];
      int pa[2], pb[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = e0 + u * kBlock;
        const int b = e / kMaxChain;
        const int a = b < Tb ? blk[b] + (e - b * kMaxChain) : b + 1;  // a > b: no pair
        pa[u] = a;
        pb[u] = b;
        if (a <= b) {
          tv[u][0] = TS[(int64_t)cols[a] * Tb + b];
          tv[u][1] = TS[(int64_t)cols[b] * Tb + a];
          tv[u][2] = S[(int64_t)cols[a] * n + cols[b]];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int a = pa[u], b = pb[u];
        if (a > b) continue;
        const int b0 = blk[b];
        const double c = (W[b * ldw + (a - b0)] + W[a * ldw + (b - b0)]) - (tv[u][0] + tv[u][1]) + tv[u][2];
        W[b * ldw + (a - b0)] = c;
        W[a * ldw + (b - b0)] = c;
      }
    }
    __syncthreads();
    // per-chain Gershgorin shift making every diagonal block positive
    // definite: each column's disc (lower end -> shift, upper end -> nrm,
    // which is rewritten after the Jacobi), then each chain's first column
    // takes the extremes over its chain
    for (int q = threadIdx.x; q < Tb; q += kBlock) {
      const int b0 = blk[q], m = bend[q] - b0;
      double sacc = 0.0;
      for (int r = 0; r < m; ++r)
        if (r != q - b0) sacc += fabs(W[q * ldw + r]);
      const double d = W[q * ldw + (q - b0)];
      shift[q] = d - sacc;
      nrm[q] = d + sacc;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < Tb; j += kBlock) {
      if (blk[j] != j) continue;
      const int e = bend[j];
      double lo = DBL_MAX, hi = -DBL_MAX;
      for (int q = j; q < e; ++q) {
        lo = fmin(lo, shift[q]);
        hi = fmax(hi, nrm[q]);
      }
      const double sh = (lo < 0.0 ? -lo : 0.0) + 0.05 * (hi - lo) + DBL_MIN;
      for (int q = j; q < e; ++q) shift[q] = sh;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < Tb; j += kBlock) W[j * ldw + (j - blk[j])] += shift[j];
    __syncthreads();
    static_assert(8 * 8 == kMaxChain && ldw >= kMaxChain, "chain columns of kMaxChain rows");
    const int sw = chain_jacobi<kBlock, 8, 8>(W, ldw, Tb, bt_start, bt_len, bt_poff, pch, s_nbt, nrm, jtol, jstop, 40,
                                              rot_flag);
    if (sw > 40 && threadIdx.x == 0) s_fail = 1;
    for (int j = threadIdx.x; j < Tb; j += kBlock) {
      double s2 = 0.0;
      for (int r = 0; r < bend[j] - blk[j]; ++r) s2 = fma(W[j * ldw + r], W[j * ldw + r], s2);
      nrm[j] = sqrt(s2);
    }
    __syncthreads();
    // Q(:, rank) = w_j/|w_j| with the rank inside the chain; eigenvalue |w_j| - shift
    for (int j = threadIdx.x; j < Tb; j += kBlock) {
      const int b0 = blk[j];
      const double lj = nrm[j] - shift[j];
      int rank = b0;
      for (int q = b0; q < bend[j]; ++q) {
        const double lq = nrm[q] - shift[q];
        rank += (lq < lj || (lq == lj && q < j)) ? 1 : 0;
      }
      src[rank] = (short)j;
      eval[it.e_off + cols[rank]] = lj;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < Tb * Tb; e += kBlock) {
      const int r = e / Tb, c = e - r * Tb, j = src[c], b0 = blk[c];
      QB[e] = (r >= b0 && r < bend[c]) ? W[j * ldw + (r - b0)] / nrm[j] : 0.0;
    }
    __syncthreads();
    // P Q -> the batch's columns of M
    for (int tm = 0; tm < nt; ++tm) {
      gemm_tile<T64>(As, Bs, tm * kTM, 0, n, Tb, Tb, row_view<double>(P, n, Tb), col_view<double>(QB, Tb, Tb), acc);
      tile_store<T64>(tm * kTM, 0, n, Tb, acc, [&](int r, int cc, double v) { M[(int64_t)r * n + cols[cc]] = v; });
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kBlock)
    if (reach[i] < 0) eval[it.e_off + i] = lam[i];
  if (threadIdx.x == 0 && s_fail && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// One-sided Jacobi on one chain matrix C (m <= G * RMAX columns of m rows,
// leading dimension ld, in LDS) for the long-chain kernel: lane groups of G
// take one column pair each, BLOCK / G >= m / 2 groups cover every pair of a
// round-robin step at once, and the squared column norms are tracked through
// the rotations (|w_p'|^2 = |w_p|^2 - t g, |w_q'|^2 = |w_q|^2 + t g with
// g = w_p.w_q) from exact values at the start of every sweep, so a pair
// costs one dot product.  nrm: m doubles of LDS.  Same skip test (cosine
// above tol), stopping rule (a sweep whose largest rotated cosine is below
// stop) and return value as chain_jacobi; ends with a barrier.  Rows m ..
// G * RMAX - 1 of every column must be zero (ld >= G * RMAX): the loads and
// stores then need no guard, and rotations keep those rows zero.
template <int BLOCK, int G, int RMAX>
__device__ __forceinline__ int long_chain_jacobi(double* C, int ld, int m, double* nrm, double tol, double stop,
                                                 int max_sweeps, int* rot_flag) {
  static_assert(BLOCK / G * 2 >= G * RMAX, "one round per step");
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  const int ne = (m + 1) & ~1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int j = grp; j < m; j += BLOCK / G) {
      const double* c = C + j * ld + lane;
      double s2 = 0.0;
#pragma unroll
      for (int k = 0; k < RMAX; ++k) s2 = fma(c[k * G], c[k * G], s2);
      s2 = group_sum<G>(s2);
      if (lane == 0) nrm[j] = s2;
    }
    __syncthreads();
    float cmax = 0.0f;
    // round-robin positions grp and ne - 1 - grp: (pos - 1 + step) mod (ne - 1)
    int vp = grp - 1, vq = ne - 2 - grp;
    for (int step = 0; step < ne - 1; ++step) {
      const int p = grp == 0 ? 0 : 1 + vp, q = 1 + vq;
      if (++vp == ne - 1) vp = 0;
      if (++vq == ne - 1) vq = 0;
      if (grp < ne / 2 && p < m && q < m) {
        double* wp = C + p * ld + lane;
        double* wq = C + q * ld + lane;
        double xp[RMAX], xq[RMAX];
        double ga0 = 0.0, ga1 = 0.0;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
          xp[k] = wp[k * G];
          xq[k] = wq[k * G];
          if (k & 1)
            ga1 = fma(xp[k], xq[k], ga1);
          else
            ga0 = fma(xp[k], xq[k], ga0);
        }
        const double ga = group_sum<G>(ga0 + ga1);
        const double al = nrm[p], be = nrm[q];
        const double cosv = fabs(ga) * rsqrt(al * be);
        if (cosv > tol) {
          // hestenes_rotation with one division (as in chain_jacobi)
          const double d = be - al, g = 2.0 * ga;
          const double t = copysign(1.0, d) * g / (fabs(d) + sqrt(fma(d, d, g * g)));
          const double cs = rsqrt(fma(t, t, 1.0)), sn = cs * t;
#pragma unroll
          for (int k = 0; k < RMAX; ++k) {
            wp[k * G] = cs * xp[k] - sn * xq[k];
            wq[k * G] = sn * xp[k] + cs * xq[k];
          }
          if (lane == 0) {
            nrm[p] = al - t * ga;
            nrm[q] = be + t * ga;
          }
          cmax = fmaxf(cmax, (float)cosv);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) cmax = fmaxf(cmax, __shfl_xor(cmax, off, 64));
    if ((threadIdx.x & 63) == 0 && cmax > 0.0f) atomicMax(&rot_flag[sweep], __float_as_int(cmax));
    __syncthreads();
    if (__int_as_float(rot_flag[sweep]) < (float)stop) return sweep + 1;
  }
  return max_sweeps + 1;
}

// ------------------------------------------------------------ long chains
// The chains of more than kMaxChain columns that refine_chain_kernel listed
// at the end of the item's W7, one work-group per item, after it on the same
// stream (items with none return at once).  Per chain i0 .. i0+m-1:
// P = (I + E)[:, chain] -> W5 (n x m), T -> Y, C = P^T S P from P^T T, a Gershgorin
// shift, the FP64 one-sided Jacobi on C, the sorted Q -> Y, P Q -> the
// chain's columns of M, eigenvalues |w_j| - shift.  C stays in LDS for
// m <= kBigLdsN (long_chain_jacobi: 64 lane groups of 4, all pairs of a
// round-robin step at once, tracked norms), above in W7 (Jacobi with lane
// groups of 64 in device memory).  Dynamic LDS: the GEMM staging tiles, overlaid by C, then the
// column norms.
constexpr int kBigLdsN = 126;
// column stride of C in LDS: 132 = 4 (mod 32) doubles, so the columns read by
// the eight 4-lane groups of a half wavefront in one round-robin step
// (consecutive indices) start 8 banks apart and cover all 64 banks
constexpr int kBigLd = 132;
constexpr int kBigDynDoubles = (2 * kTileLds > kBigLdsN * kBigLd ? 2 * kTileLds : kBigLdsN * kBigLd) + kMaxN;
__global__ __launch_bounds__(kBlock) void refine_bigchain_kernel(const ItemDev* __restrict__ items,
                                                                 const double* __restrict__ lam_pre,
                                                                 double* __restrict__ eval, double* work,
                                                                 int32_t* __restrict__ status, double closec,
                                                                 double jtol, double jstop) {
  extern __shared__ double bsm[];
  double* const As = bsm;
  double* const Bs = bsm + kTileLds;
  double* const bnrm = bsm + (kBigDynDoubles - kMaxN);
  __shared__ double lam[kMaxN];
  __shared__ short big_start[kMaxBig], big_len[kMaxBig];
  __shared__ int rot_flag[64];
  __shared__ double s_lo[kBlock / 64], s_hi[kBlock / 64];
  __shared__ int s_nbig, s_fail;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  if (n <= kMaxChain) return;  // no chain can be longer than kMaxChain
  const WS ws(work, it);
  if (threadIdx.x == 0) {
    const double* tail = ws.W7 + (int64_t)n * n - (2 * kMaxBig + 1);
    s_nbig = (int)tail[0];
    for (int b = 0; b < s_nbig; ++b) {
      big_start[b] = (short)tail[1 + 2 * b];
      big_len[b] = (short)tail[2 + 2 * b];
    }
    s_fail = 0;
  }
  __syncthreads();
  if (s_nbig == 0) return;
  for (int i = threadIdx.x; i < n; i += kBlock) lam[i] = lam_pre[it.e_off + i];
  __syncthreads();
  const double* S = ws.S;
  const double* G = ws.G;
  double* P = ws.W5;
  double* TS = ws.Y;  // T = S_C + Lam E / 2
  double* Q = ws.Y;   // after T's last use
  double* M = ws.W6;
  const int nt = (n + kTM - 1) / kTM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  d4 acc[2][2];
  for (int b = 0; b < s_nbig; ++b) {
    const int i0 = big_start[b], m = big_len[b];
    const int mt = (m + kTM - 1) / kTM;
    const bool in_lds = m <= kBigLdsN;
    double* const C = in_lds ? bsm : ws.W7;  // C overlays the staging tiles in LDS
    const int ld = in_lds ? kBigLd : m;
    for (int e = threadIdx.x; e < n * m; e += kBlock) {
      const int k = e / m, t = e - k * m;
      const int64_t ue = upper_at(n, k, i0 + t);
      const double sv = S[ue];
      const double ek = newton_e_of(G[ue], sv, lam[k], lam[i0 + t], k == i0 + t, closec);
      P[e] = (k == i0 + t ? 1.0 : 0.0) + ek;
      TS[e] = fma(0.5 * lam[k], ek, sv);
    }
    __syncthreads();
    // V = P^T T (every tile: V is not symmetric) -> C as it is
    auto put_c = [&](int r, int cc, double v) { C[cc * ld + r] = v; };
    if (in_lds) {
      // m <= 126: the 2 x 2 tiles of V are all computed before any is
      // stored, since C overlays the staging tiles
      static_assert(kBigLdsN <= 2 * kTM && kBigLd >= 128, "at most 2 x 2 tiles of C in LDS, 128 rows per column");
      d4 acc4[4][2][2];
      const auto pv = col_view<double>(P, n, m);
      const auto tv = col_view<double>(TS, n, m);
      gemm_tile<T64>(As, Bs, 0, 0, m, m, n, pv, tv, acc4[0]);
      if (mt > 1) {
        gemm_tile<T64>(As, Bs, 0, kTM, m, m, n, pv, tv, acc4[1]);
        gemm_tile<T64>(As, Bs, kTM, 0, m, m, n, pv, tv, acc4[2]);
        gemm_tile<T64>(As, Bs, kTM, kTM, m, m, n, pv, tv, acc4[3]);
      }
      __syncthreads();
      tile_store<T64>(0, 0, m, m, acc4[0], put_c);
      if (mt > 1) {
        tile_store<T64>(0, kTM, m, m, acc4[1], put_c);
        tile_store<T64>(kTM, 0, m, m, acc4[2], put_c);
        tile_store<T64>(kTM, kTM, m, m, acc4[3], put_c);
      }
    } else {
      for (int tm = 0; tm < mt; ++tm)
        for (int tc = 0; tc < mt; ++tc) {
          gemm_tile<T64>(As, Bs, tm * kTM, tc * kTM, m, m, n, col_view<double>(P, n, m), col_view<double>(TS, n, m),
                         acc);
          tile_store<T64>(tm * kTM, tc * kTM, m, m, acc, put_c);
        }
    }
    __syncthreads();
    // P^T S P ~ V + V^T - T_C - T_C^T + S_CC, one thread per pair a <= b;
    // the loads of four pairs are issued before any is used
    for (int e0 = threadIdx.x; e0 < m * m; e0 += 4 * kBlock) {
      double tv[4][3];
      int pa[4], pb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kBlock;
        const int b = e / m;
        const int a = b < m ? e - b * m : b + 1;  // a > b: no pair
        pa[u] = a;
        pb[u] = b;
        if (a <= b) {
          tv[u][0] = TS[(int64_t)(i0 + a) * m + b];
          tv[u][1] = TS[(int64_t)(i0 + b) * m + a];
          tv[u][2] = S[(int64_t)(i0 + a) * n + i0 + b];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = pa[u], b = pb[u];
        if (a > b) continue;
        const double c = (C[b * ld + a] + C[a * ld + b]) - (tv[u][0] + tv[u][1]) + tv[u][2];
        C[b * ld + a] = c;
        C[a * ld + b] = c;
      }
    }
    if (threadIdx.x < 64) rot_flag[threadIdx.x] = 0;
    __syncthreads();
    // Gershgorin shift: one wavefront per column
    double lo = DBL_MAX, hi = -DBL_MAX;
    for (int q = wave; q < m; q += kBlock / 64) {
      double sacc = 0.0;
      for (int r = lane; r < m; r += 64) sacc += (r == q) ? 0.0 : fabs(C[q * ld + r]);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
      const double d = C[q * ld + q];
      lo = fmin(lo, d - sacc);
      hi = fmax(hi, d + sacc);
    }
    if (lane == 0) {
      s_lo[wave] = lo;
      s_hi[wave] = hi;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    for (int w = 1; w < kBlock / 64; ++w) {
      lo = fmin(lo, s_lo[w]);
      hi = fmax(hi, s_hi[w]);
    }
    const double sh = (lo < 0.0 ? -lo : 0.0) + 0.05 * (hi - lo) + DBL_MIN;
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += kBlock) C[j * ld + j] += sh;
    // in LDS: rows m .. 127 of every column zero (long_chain_jacobi reads and
    // writes them unguarded)
    if (in_lds)
      for (int e = threadIdx.x; e < m * (128 - m); e += kBlock) {
        const int j = e / (128 - m);
        bsm[j * kBigLd + m + (e - j * (128 - m))] = 0.0;
      }
    __syncthreads();
    const int swb = in_lds ? long_chain_jacobi<kBlock, 4, 32>(bsm, kBigLd, m, bnrm, jtol, jstop, 40, rot_flag)
                           : onesided_jacobi_lds<double, kBlock, 64, kBigRows>(C, m, m, 1e-15, 8e-15, 40, rot_flag);
    if (swb > 40 && threadIdx.x == 0) s_fail = 1;
    for (int j = wave; j < m; j += kBlock / 64) {
      double s2 = 0.0;
      for (int r = lane; r < m; r += 64) s2 = fma(C[j * ld + r], C[j * ld + r], s2);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s2 += __shfl_xor(s2, off, 64);
      if (lane == 0) bnrm[j] = sqrt(s2);
    }
    __syncthreads();
    // sorted Q (Q[r][rank] = w_j[r]/|w_j|) -> Y; eigenvalue |w_j| - shift
    for (int j = wave; j < m; j += kBlock / 64) {
      const double lj = bnrm[j];
      int cnt = 0;
      for (int q = lane; q < m; q += 64) cnt += (bnrm[q] < lj || (bnrm[q] == lj && q < j)) ? 1 : 0;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
      for (int r = lane; r < m; r += 64) Q[(int64_t)r * m + cnt] = C[j * ld + r] / lj;
      if (lane == 0) eval[it.e_off + i0 + cnt] = lj - sh;
    }
    __syncthreads();
    for (int tm = 0; tm < nt; ++tm)
      for (int tc = 0; tc < mt; ++tc) {
        gemm_tile<T64>(As, Bs, tm * kTM, tc * kTM, n, m, m, row_view<double>(P, n, m), col_view<double>(Q, m, m), acc);
        tile_store<T64>(tm * kTM, tc * kTM, n, m, acc,
                        [&](int r, int cc, double v) { M[(int64_t)r * n + i0 + cc] = v; });
      }
    __syncthreads();
  }
  if (threadIdx.x == 0 && s_fail && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// ------------------------------------------------------------ finish
// Sort the eigenpairs by eigenvalue (ties by index) and write them to the
// caller's arrays; X is read from the work-space (x_ws) or from evec (then
// staged through Y when a permutation is needed).
__global__ __launch_bounds__(kBlock) void refine_finish_kernel(const ItemDev* __restrict__ items, double* evec,
                                                               int x_ws, double* work, double* __restrict__ eval,
                                                               int32_t* __restrict__ status) {
  __shared__ double lam[kMaxN];
  __shared__ int rank[kMaxN];
  __shared__ int s_perm, s_bad;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  const WS ws(work, it);
  double* ev = eval + it.e_off;
  double* X = evec + it.v_off;
  if (threadIdx.x == 0) {
    s_perm = 0;
    s_bad = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    lam[i] = ev[i];
    if (!isfinite(lam[i])) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    int r = 0;
    for (int q = 0; q < n; ++q) r += (lam[q] < lam[i] || (lam[q] == lam[i] && q < i)) ? 1 : 0;
    rank[i] = r;
    if (r != i) atomicOr(&s_perm, 1);
  }
  __syncthreads();
  const int64_t nn = (int64_t)n * n;
  const double* src = X;
  if (x_ws) {
    src = ws.P1;
  } else if (s_perm) {
    for (int64_t e = threadIdx.x; e < nn; e += kBlock) ws.Y[e] = X[e];
    __syncthreads();
    src = ws.Y;
  }
  if (x_ws || s_perm) {
    for (int64_t e = threadIdx.x; e < nn; e += kBlock) {
      const int r = (int)(e / n), c = (int)(e - (int64_t)r * n);
      X[(int64_t)r * n + rank[c]] = src[e];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) ev[rank[i]] = lam[i];
  if (threadIdx.x == 0 && s_bad && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// Ranks of the refined eigenvalues (ties by index) -> cl, eval sorted in
// place, a non-finite eigenvalue flagged; the last step's X M then writes
// every eigenvector straight to its sorted column (whole-item products).
__global__ __launch_bounds__(kBlock) void refine_rank_kernel(const ItemDev* __restrict__ items,
                                                             double* __restrict__ eval, int32_t* __restrict__ cl,
                                                             int32_t* __restrict__ status) {
  __shared__ double lam[kMaxN];
  __shared__ int rank[kMaxN];
  __shared__ int s_bad;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  double* ev = eval + it.e_off;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    lam[i] = ev[i];
    if (!isfinite(lam[i])) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    int r = 0;
    for (int q = 0; q < n; ++q) r += (lam[q] < lam[i] || (lam[q] == lam[i] && q < i)) ? 1 : 0;
    rank[i] = r;
    cl[it.e_off + i] = r;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) ev[rank[i]] = lam[i];
  if (threadIdx.x == 0 && s_bad && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// ------------------------------------------------- FP64 Jacobi epilogue
// Y = H X for the normalised columns of the device-memory FP64 Jacobi (column
// c of X contiguous at ws.P1 + c n, as the iteration stores W); Y column-major
// in ws.Y.
__global__ __launch_bounds__(T64::NT, 3) void rq_hx_kernel(const ItemDev* __restrict__ items, int n_items,
                                                         const GridDev* __restrict__ grids,
                                                         const double* __restrict__ v64, double* work, int tiles) {
  WPCD_LDS_TILES(T64, 1);
  int item, tile;
  if (!xcd_item_tile(tiles, n_items, item, tile)) return;
  const ItemDev it = items[item];
  const int n = it.n;
  const int nt = (n + T64::TM - 1) / T64::TM;
  if (tile >= nt * nt) return;
  const int tm = tile / nt, tc = tile % nt;
  const GridDev g = grids[it.grid];
  const WS ws(work, it);
  const double* X = ws.P1;
  d4 acc[2][2];
  // B(k, j) = component k of column j = X[j n + k]
  gemm_tile<T64>(As, Bs, tm * T64::TM, tc * T64::TM, n, n, n, col_view(v64 + it.v_off, n, n), row_view<double>(X, n, n), acc);
  double* Y = ws.Y;
  const int N = it.N;
  tile_store<T64>(tm * T64::TM, tc * T64::TM, n, n, acc, [&](int r, int c, double v) {
    Y[(int64_t)c * n + r] = fma(g.e0[r % N], X[(int64_t)c * n + r], v);  // + H0 X
  });
}

// lambda_c = x_c . (H x_c) / x_c . x_c, ranked ascending (ties by index);
// eval[rank] = lambda, evec[r][rank] = x_c[r].  One work-group per item.
__global__ __launch_bounds__(kBlock) void rq_sort_kernel(const ItemDev* __restrict__ items, const double* work,
                                                        double* __restrict__ evec, double* __restrict__ eval,
                                                        int32_t* __restrict__ status) {
  __shared__ double lam[kMaxN];
  __shared__ int rank[kMaxN];
  __shared__ int s_bad;
  const ItemDev it = items[blockIdx.x];
  const int n = it.n;
  const double* X = work + it.w_off;
  const double* Y = X + (int64_t)n * n;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < n; c += kBlock / 64) {
    double q = 0.0, vv = 0.0;
    for (int r = lane; r < n; r += 64) {
      const double x = X[(int64_t)c * n + r];
      q = fma(x, Y[(int64_t)c * n + r], q);
      vv = fma(x, x, vv);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      q += __shfl_xor(q, off, 64);
      vv += __shfl_xor(vv, off, 64);
    }
    if (lane == 0) {
      const double l = q / vv;
      lam[c] = l;
      if (!isfinite(l)) s_bad = 1;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kBlock) {
    const double lc = lam[c];
    int k = 0;
    for (int i = 0; i < n; ++i) k += (lam[i] < lc || (lam[i] == lc && i < c)) ? 1 : 0;
    rank[c] = k;
  }
  __syncthreads();
  double* E = evec + it.v_off;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kBlock) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    E[(int64_t)r * n + rank[c]] = X[e];
  }
  for (int c = threadIdx.x; c < n; c += kBlock) eval[it.e_off + rank[c]] = lam[c];
  if (threadIdx.x == 0 && s_bad && status[blockIdx.x] >= 0) status[blockIdx.x] = WPCD_ERR_NUMERIC;
}

// ------------------------------------------------ LDS Jacobi warm start
// Reference eigenvectors (x32: row-major, ascending) -> Q0 with columns in
// descending eigenvalue order, column-major floats at the reference's
// work-space (free until the refinement).  One work-group per reference.
__global__ __launch_bounds__(kBlock) void warm_q0_kernel(const ItemDev* __restrict__ items,
                                                        const int32_t* __restrict__ refs,
                                                        const float* __restrict__ x32, double* work) {
  const ItemDev it = items[refs[blockIdx.x]];
  const int n = it.n;
  const float* X = x32 + it.v_off;
  float* Q0 = reinterpret_cast<float*>(work + it.w_off);
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kBlock) {
    const int j = (int)(e / n), r = (int)(e - (int64_t)j * n);
    Q0[e] = X[(int64_t)r * n + (n - 1 - j)];
  }
}

// Reference choice of the warm starts.  The iteration from W = B Q0 needs
// fewer sweeps the closer the reference's H is to the item's (a NumPy model
// of the coupled batch: 3.1 instead of 3.8 sweeps when the nearest of 64
// cold items in Frobenius norm replaces the first one), and a strided sample
// of kWarmSig entries of V picks the same nearest item there.
// Sample of V per item: entry s * stride, stride = n^2 / min(n^2, kWarmSig)
// (all entries of small items; zero-filled to kWarmSig).  One work-group per
// item of the batch.
__global__ __launch_bounds__(kBlock) void warm_sig_kernel(const ItemDev* __restrict__ items,
                                                         const double* __restrict__ v64, float* __restrict__ sig) {
  const ItemDev it = items[blockIdx.x];
  const int64_t nn = (int64_t)it.n * it.n;
  const int cnt = nn < kWarmSig ? (int)nn : kWarmSig;
  const int64_t stride = nn / cnt;
  float* out = sig + (int64_t)blockIdx.x * kWarmSig;
  for (int q = threadIdx.x; q < kWarmSig; q += kBlock) out[q] = q < cnt ? (float)v64[it.v_off + q * stride] : 0.0f;
}

// One work-group per pick task: the task's warm items' samples in LDS, the
// threads over the group's candidates, squared distances of the samples; the
// nearest candidate (ties: the earlier in the list) becomes the reference.
__global__ __launch_bounds__(kBlock) void warm_pick_kernel(const int32_t* __restrict__ pick,
                                                          const int32_t* __restrict__ jlist,
                                                          const int32_t* __restrict__ cand,
                                                          const float* __restrict__ sig, int32_t* __restrict__ ref) {
  __shared__ float4 ws[kWarmPick][kWarmSig / 4];
  __shared__ float rd[kBlock / 64][kWarmPick];
  __shared__ int ri[kBlock / 64][kWarmPick];
  const int woff = pick[4 * blockIdx.x], wcnt = pick[4 * blockIdx.x + 1];
  const int coff = pick[4 * blockIdx.x + 2], ccnt = pick[4 * blockIdx.x + 3];
  for (int e = threadIdx.x; e < kWarmPick * kWarmSig / 4; e += kBlock) {
    const int w = e / (kWarmSig / 4), q = e - w * (kWarmSig / 4);
    ws[w][q] = w < wcnt ? reinterpret_cast<const float4*>(sig + (int64_t)jlist[woff + w] * kWarmSig)[q]
                        : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  __syncthreads();
  float best[kWarmPick];
  int bi[kWarmPick];
#pragma unroll
  for (int w = 0; w < kWarmPick; ++w) {
    best[w] = INFINITY;
    bi[w] = 0x7fffffff;
  }
  for (int c = threadIdx.x; c < ccnt; c += kBlock) {
    const float4* sc = reinterpret_cast<const float4*>(sig + (int64_t)cand[coff + c] * kWarmSig);
    float d[kWarmPick];
#pragma unroll
    for (int w = 0; w < kWarmPick; ++w) d[w] = 0.0f;
    for (int q4 = 0; q4 < kWarmSig / 4; ++q4) {
      const float4 x = sc[q4];
#pragma unroll
      for (int w = 0; w < kWarmPick; ++w) {
        const float4 y = ws[w][q4];
        const float a = y.x - x.x, b = y.y - x.y, cc = y.z - x.z, dd = y.w - x.w;
        d[w] = fmaf(a, a, fmaf(b, b, fmaf(cc, cc, fmaf(dd, dd, d[w]))));
      }
    }
#pragma unroll
    for (int w = 0; w < kWarmPick; ++w)
      if (d[w] < best[w]) {  // c grows per thread: ties keep the earlier candidate
        best[w] = d[w];
        bi[w] = c;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < kWarmPick; ++w) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const float od = __shfl_xor(best[w], off, 64);
      const int oi = __shfl_xor(bi[w], off, 64);
      if (od < best[w] || (od == best[w] && oi < bi[w])) {
        best[w] = od;
        bi[w] = oi;
      }
    }
    if (lane == 0) {
      rd[wave][w] = best[w];
      ri[wave][w] = bi[w];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < wcnt) {
    const int w = threadIdx.x;
    float bd = rd[0][w];
    int bx = ri[0][w];
    for (int v = 1; v < kBlock / 64; ++v)
      if (rd[v][w] < bd || (rd[v][w] == bd && ri[v][w] < bx)) {
        bd = rd[v][w];
        bx = ri[v][w];
      }
    if (bx < ccnt) ref[jlist[woff + w]] = cand[coff + bx];
  }
}

// H Q0 for every warm item (its reference's Q0), column-major FP32 into the
// item's x32, where the Jacobi kernel reads it as the start of W.  The result
// only seeds an FP32 iteration, so the product runs on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, D[i][j] in lane j + 16 (i / 4), register i % 4) with 64 x 64 tiles
// of 4 wavefronts (32 x 32 each) and K chunks of 32; staged tiles are
// T[k * 64 + (i ^ 16 (k % 4))] floats, so the 4 k of an operand read land in
// 4 distinct 16-bank ranges and the stores (64 lanes over i) in all 64.
typedef float f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(T64::NT, 3) void warm_y_kernel(const ItemDev* __restrict__ items,
                                                           const int32_t* __restrict__ warm, int n_warm,
                                                           const int32_t* __restrict__ ref,
                                                           const GridDev* __restrict__ grids,
                                                           const double* __restrict__ v64, float* x32,
                                                           const double* work, int tiles) {
  __shared__ float As[kTK * 64];
  __shared__ float Bs[kTK * 64];
  int w, tile;
  if (!xcd_item_tile(tiles, n_warm, w, tile)) return;
  const int item = warm[w];
  const ItemDev it = items[item];
  const int n = it.n;
  const int nt = (n + 63) / 64;
  if (tile >= nt * nt) return;
  const int m0 = (tile / nt) * 64, c0 = (tile % nt) * 64;
  const GridDev g = grids[it.grid];
  const float* Q0 = reinterpret_cast<const float*>(work + items[ref[item]].w_off);
  const Mat<double> A = col_view(v64 + it.v_off, n, n);  // A(i, k) = V[k][i] = V[i][k]
  const Mat<float> B = row_view<float>(Q0, n, n);        // B(k, j) = Q0[j n + k]
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // staging map: thread t loads i = t % 64 and k = 4 (t / 64 + 4h) + j
  const int si = tid & 63, sg = wave;
  Mat<double>::raw_t ra[8];
  Mat<float>::raw_t rb[8];
  auto load = [&](int k0) {
    const unsigned ba = m0 + si < n ? (unsigned)((m0 + si) * A.si) * 8u : kOob;
    const unsigned bb = c0 + si < n ? (unsigned)((c0 + si) * B.si) * 4u : kOob;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * (sg + 4 * h) + j;
        ra[4 * h + j] = A.load(ba + (k < n ? (unsigned)(k * A.sk) * 8u : kOob));
        rb[4 * h + j] = B.load(bb + (k < n ? (unsigned)(k * B.sk) * 4u : kOob));
      }
  };
  f4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
  const int kk = lane >> 4, sw = kk << 4;  // k % 4 = lane / 16 for k = 4q + lane / 16
  const int pa[2] = {kk * 64 + ((wr + (lane & 15)) ^ sw), kk * 64 + ((wr + 16 + (lane & 15)) ^ sw)};
  const int pb[2] = {kk * 64 + ((wc + (lane & 15)) ^ sw), kk * 64 + ((wc + 16 + (lane & 15)) ^ sw)};
  load(0);
  for (int k0 = 0; k0 < n; k0 += kTK) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * (sg + 4 * h) + j;
        As[k * 64 + (si ^ ((k & 3) << 4))] = (float)Mat<double>::cvt(ra[4 * h + j]);
        Bs[k * 64 + (si ^ ((k & 3) << 4))] = (float)Mat<float>::cvt(rb[4 * h + j]);
      }
    __syncthreads();
    if (k0 + kTK < n) load(k0 + kTK);
    const int qend = (n - k0) < kTK ? (n - k0 + 3) >> 2 : kTK / 4;
    for (int q = 0; q < qend; ++q) {
      const int o = q * 256;
      const float a0 = As[o + pa[0]], a1 = As[o + pa[1]], b0 = Bs[o + pb[0]], b1 = Bs[o + pb[1]];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  float* Y0 = x32 + it.v_off;
  const int N = it.N;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int c = c0 + wc + bj * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = m0 + wr + bi * 16 + 4 * (lane >> 4) + rr;
        if (r < n && c < n) Y0[(int64_t)c * n + r] = fmaf((float)g.e0[r % N], Q0[(int64_t)c * n + r], acc[bi][bj][rr]);
      }
    }
}

// ------------------------------------ whole-item products (193 <= n <= 208)
// For items of 193..208 rows (13 x 13 output blocks of 16 x 16) one
// work-group of 12 wavefronts computes a whole n x n product, in two passes
// over K.  Wavefront w owns row strip w of the blocks, and the 13 blocks of
// strip 12 are shared out:
//   general products: pass 0 the columns 0..6, plus (12, w) for w < 7;
//                     pass 1 the columns 7..12, plus (12, w) for w >= 7 and,
//                     for w = 0, (12, 12);
//   symmetric products (one block per unordered pair, stored mirrored; the
//                     two passes are two products): columns (w + j) mod 13,
//                     j < 7, plus (12, (12 + w) mod 13) for w < 7.
// Each SIMD (wavefronts s, s + 4, s + 8) then carries 22-23 and 19-20 blocks
// in the two passes of a general product, 22-23 per symmetric one, and no
// wavefront holds more than 8 accumulator blocks.  K is staged in chunks of
// 16 as panels in LDS: the A panel over all 208 rows, the B panel over the
// pass's columns only, so both MFMA operands of every block come from LDS;
// the B panel is fetched once per item and the A panel once per pass
// (64 x 64 tiles fetch each panel four times).  The work-groups are
// persistent, one per CU, and load the next chunk -- of the same pass, of
// the next pass or of their next item -- into registers while the current
// one is multiplied; LDS holds two chunks, one barrier per chunk.
// Panel layouts: a source contiguous along i (a column view) is staged
// k-major, element (i, k) at P[k * 208 + i]: the stores cover consecutive i,
// and an MFMA read (16 lanes over i at k and at k + 1 in one half wavefront)
// puts k + 1 416 four-byte banks = half of the banks away.  A source
// contiguous along k (a row view) is staged i-major, P[i * 18 + k]: the loads
// cover 16 consecutive k of 4 rows (128-byte segments), and the 16 rows of an
// MFMA read start 36 banks apart, so rows at k and k + 1 touch all 64 banks.
constexpr int kIW = 12;                  // wavefronts (3 per SIMD)
constexpr int kIT = 64 * kIW;            // threads
constexpr int kIKC = 16;                 // K chunk
constexpr int kIN = 208;                 // largest n
constexpr int kINMin = 193;              // smallest n (13 block rows)
constexpr int kIBlk = kIN / 16;          // blocks per side
constexpr int kILdI = kIKC + 2;          // row stride of an i-major panel
constexpr int kIPanelLds = kIN * kILdI;  // LDS doubles per panel (either layout)
static_assert(kIBlk == kIW + 1, "one row strip per wavefront plus one shared strip");

// staging of the panel rows [I0, I0 + W) of one K chunk: ceil(16 W / kIT)
// elements per thread; the last round covers whole wavefronts
template <int W>
struct IStage {
  static constexpr int E = W * kIKC;
  static constexpr int NS = (E + kIT - 1) / kIT;
  static constexpr int LAST = E - kIT * (NS - 1);
  static_assert(LAST % 64 == 0, "the last staging round must cover whole wavefronts");
};
constexpr int kIStage = IStage<kIN>::NS;  // the largest

template <bool KMAJ, int W, int I0, typename T>
__device__ __forceinline__ void ifetch(typename Mat<T>::raw_t (&r)[kIStage], const Mat<T>& m, int k0, int n) {
  using S = IStage<W>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < S::NS; ++s) {
    if (s < S::NS - 1 || tid < S::LAST) {
      const int e = tid + kIT * s;
      int i, k;
      if constexpr (KMAJ) {
        k = e / W;
        i = I0 + e - k * W;
      } else {
        static_assert(W == kIN && I0 == 0, "i-major panels span all rows");
        i = e / kIKC;
        k = e - i * kIKC;
      }
      k += k0;
      r[s] = m.load(i < n && k < n ? (unsigned)(i * m.si + k * m.sk) * (unsigned)sizeof(T) : kOob);
    }
  }
}
// dg (k-major panels only): LDS table added to the diagonal elements
// (i = k < n) of the chunk starting at k0, or nullptr
template <bool KMAJ, int W, int I0, typename T>
__device__ __forceinline__ void istash(double* P, const typename Mat<T>::raw_t (&r)[kIStage], const double* dg = nullptr,
                                       int k0 = 0, int n = 0) {
  using S = IStage<W>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < S::NS; ++s) {
    if (s < S::NS - 1 || tid < S::LAST) {
      const int e = tid + kIT * s;
      if constexpr (KMAJ) {
        const int k = e / W, i = I0 + e - k * W;
        double v = Mat<T>::cvt(r[s]);
        if (dg != nullptr && i == k0 + k && i < n) v += dg[i];
        P[k * kIN + i] = v;
      } else {
        P[(e / kIKC) * kILdI + e % kIKC] = Mat<T>::cvt(r[s]);
      }
    }
  }
}
// offset of block row/column b (16 rows) and of k step q in a panel
template <bool KMAJ>
__device__ __forceinline__ constexpr int ipan_blk(int b) { return KMAJ ? b * 16 : b * 16 * kILdI; }
template <bool KMAJ>
__device__ __forceinline__ constexpr int ipan_kstep(int q) { return KMAJ ? 4 * q * kIN : 4 * q; }

// block sets of a pass (above)
enum { kSetLo = 0, kSetHi = 1, kSetSym = 2 };
// result stores: row-major FP64 or FP32 (out<pass>() gives the buffer),
// symmetric FP64 (mirrored), or per element through store<pass>()
enum { kOutF64 = 0, kOutF32 = 1, kOutSym = 2, kOutCall = 3 };
template <int SET>
struct IBlocks {
  static constexpr int NC = SET == kSetHi ? 6 : 7;           // blocks of the own strip
  static constexpr int BC0 = SET == kSetHi ? 7 : 0;          // first staged B column block
  static constexpr int BW = SET == kSetSym ? kIBlk : NC;     // staged B column blocks
  __device__ static int col(int w, int j) { return SET == kSetSym ? (w + j) % kIBlk : BC0 + j; }
  __device__ static bool e_live(int w) { return SET == kSetHi ? w >= 7 : w < 7; }  // block (12, ce)
  __device__ static int ce(int w) { return SET == kSetSym ? (kIBlk - 1 + w) % kIBlk : w; }
  __device__ static bool x_live(int w) { return SET == kSetHi && w == 0; }         // block (12, 12)
};

// A problem P: element types TA/TB and layouts KA/KB of the A and B sources
// (A = viewA(item) in every pass, B = viewB<pass>(item) unless
// same_panel<pass>(), then B is the A panel), the block set of each pass,
// and store<pass>(item, row, col, value).
template <class P, int PS>
__device__ __forceinline__ void ifetch_pass(typename Mat<typename P::TA>::raw_t (&ra)[kIStage],
                                            typename Mat<typename P::TB>::raw_t (&rb)[kIStage], const P& p,
                                            const ItemDev& it, int item, int k0) {
  using B = IBlocks<P::set(PS)>;
  ifetch<P::KA, kIN, 0>(ra, p.viewA(it, item), k0, it.n);
  if constexpr (!P::same_panel(PS))
    ifetch<P::KB, B::BW * 16, B::BC0 * 16>(rb, p.template viewB<PS>(it, item), k0, it.n);
}

template <class P, int PS>
__device__ __forceinline__ void ipass(const P& p, const ItemDev* __restrict__ items, const int32_t* sel,
                                      int n_items, int i, int item, const ItemDev& it,
                                      double (*lds)[2][kIPanelLds], double* dg, int* pm, int& buf,
                                      typename Mat<typename P::TA>::raw_t (&ra)[kIStage],
                                      typename Mat<typename P::TB>::raw_t (&rb)[kIStage]) {
  using B = IBlocks<P::set(PS)>;
  constexpr bool SAME = P::same_panel(PS);
  constexpr bool KB = SAME ? P::KA : P::KB;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int loa = P::KA ? lk * kIN + li : li * kILdI + lk;
  const int lob = KB ? lk * kIN + li : li * kILdI + lk;
  const int oa = loa + ipan_blk<P::KA>(w), oa12 = loa + ipan_blk<P::KA>(kIBlk - 1);
  int ob[B::NC];
#pragma unroll
  for (int j = 0; j < B::NC; ++j) ob[j] = lob + ipan_blk<KB>(B::col(w, j));
  const int obe = lob + ipan_blk<KB>(B::ce(w)), obx = lob + ipan_blk<KB>(kIBlk - 1);
  const bool e_live = B::e_live(w), x_live = B::x_live(w);
  const int n = it.n;
  d4 acc[B::NC], ace = {0.0, 0.0, 0.0, 0.0}, acx = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < B::NC; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  const int nck = (n + kIKC - 1) / kIKC;
  if constexpr (P::DIAG_A || P::DIAG_B) {
    // the diagonal added to A or B; every wavefront has passed the last
    // barrier of the previous item, so none still stages from the old table
    if (PS == 0) {
      for (int i = threadIdx.x; i < n; i += kIT) dg[i] = p.diag(it, i);
      __syncthreads();
    }
  }
  if constexpr (P::PERM) {
    // output column permutation (read in the epilogues: wait until the
    // previous item's are done)
    if (PS == 0 && p.perm != nullptr) {
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kIT) pm[i] = p.perm[it.e_off + i];
      __syncthreads();
    }
  }
  for (int c = 0; c < nck; ++c) {
    double* const LA = lds[buf][0];
    double* const LB = SAME ? LA : lds[buf][1];
    istash<P::KA, kIN, 0, typename P::TA>(LA, ra, P::DIAG_A ? dg : nullptr, c * kIKC, n);
    if constexpr (!SAME) istash<KB, B::BW * 16, B::BC0 * 16, typename P::TB>(LB, rb, P::DIAG_B ? dg : nullptr, c * kIKC, n);
    __syncthreads();
    if (c + 1 < nck) {
      ifetch_pass<P, PS>(ra, rb, p, it, item, (c + 1) * kIKC);
    } else if constexpr (PS + 1 < P::NPASS) {
      ifetch_pass<P, (PS + 1 < P::NPASS ? PS + 1 : 0)>(ra, rb, p, it, item, 0);
    } else if (i + (int)gridDim.x < n_items) {
      const int nx = sel ? sel[i + gridDim.x] : i + gridDim.x;
      ifetch_pass<P, 0>(ra, rb, p, items[nx], nx, 0);
    }
    const int qn = (n - c * kIKC + 3) >> 2 < kIKC / 4 ? (n - c * kIKC + 3) >> 2 : kIKC / 4;
#pragma unroll 1
    for (int q = 0; q < qn; ++q) {
      const double a = LA[oa + ipan_kstep<P::KA>(q)];
      const double* const Lq = LB + ipan_kstep<KB>(q);
#pragma unroll
      for (int j = 0; j < B::NC; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Lq[ob[j]], acc[j], 0, 0, 0);
    }
    if (e_live || x_live) {
#pragma unroll 1
      for (int q = 0; q < qn; ++q) {
        const double a = LA[oa12 + ipan_kstep<P::KA>(q)];
        const double* const Lq = LB + ipan_kstep<KB>(q);
        if (e_live) ace = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Lq[obe], ace, 0, 0, 0);
        if (x_live) acx = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Lq[obx], acx, 0, 0, 0);
      }
    }
    buf ^= 1;
  }
  auto put = [&](const d4& v, int br, int bc) {
    const int col = bc * 16 + li;
    const double e[4] = {v[0], v[1], v[2], v[3]};  // (a bit_cast of v[r] itself stored v[0] four times)
    if constexpr (P::OUT == kOutF64 || P::OUT == kOutF32) {
      // row-major n x n result through buffer stores: a column past n goes
      // to an offset past the buffer, a row past n lands past it too, and
      // both are dropped
      constexpr unsigned SZ = P::OUT == kOutF64 ? 8u : 4u;
      const __amdgpu_buffer_rsrc_t o = p.template out<PS>(it, item);
      int pc = col;
      if constexpr (P::PERM)
        if (p.perm != nullptr && col < n) pc = pm[col];
      const unsigned vo = col < n ? (unsigned)((br * 16 + lk) * n + pc) * SZ : kOob;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (P::OUT == kOutF64)
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, e[r]), o, vo + (unsigned)(4 * r * n) * SZ,
                                                0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)e[r]), o,
                                                vo + (unsigned)(4 * r * n) * SZ, 0, 0);
      }
    } else if constexpr (P::OUT == kOutSym) {
      // symmetric result: only the upper triangle is stored, element (row,
      // col) at (min, max); in a diagonal block only row <= col is kept;
      // dropped stores get an offset past the buffer
      const __amdgpu_buffer_rsrc_t o = p.template out<PS>(it, item);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = br * 16 + lk + 4 * r;
        const bool keep = row < n && col < n && !(br == bc && row > col);
        const unsigned ou = !keep ? kOob : row <= col ? (unsigned)(row * n + col) * 8u : (unsigned)(col * n + row) * 8u;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, e[r]), o, ou, 0, 0);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = br * 16 + lk + 4 * r;
        if (row < n && col < n) p.template store<PS>(it, item, br == bc, row, col, e[r]);
      }
    }
  };
#pragma unroll
  for (int j = 0; j < B::NC; ++j) put(acc[j], w, B::col(w, j));
  if (e_live) put(ace, kIBlk - 1, B::ce(w));
  if (x_live) put(acx, kIBlk - 1, kIBlk - 1);
  if constexpr (P::REACH) {
    // after G (the second pass of the symmetric S, G product): the work of
    // refine_reach_kernel from the G blocks in registers and the S elements
    // this lane stored in the first pass (same blocks, same positions).
    // Rayleigh quotients lam_i = S_ii / G_ii -> dg; per row p the largest
    // close q > p (else p) -> pm; then both to lam_pre and cl.  dg and pm are
    // last read after the previous item's passes (their chunk barriers).
    if (PS == 1) {
      static_assert(P::set(PS) == kSetSym, "close-pair test on the symmetric product");
      const double* S = WS(p.work, it).S;
      auto diag_lam = [&](const d4& v, int b) {
        const double e[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = b * 16 + lk + 4 * r, col = b * 16 + li;
          if (row == col && row < n) dg[row] = S[(int64_t)row * n + row] / e[r];
        }
      };
      diag_lam(acc[0], w);  // block (w, w): column block (w + 0) mod 13
      if (w == 0 && e_live) diag_lam(ace, kIBlk - 1);  // block (12, 12)
      for (int i = threadIdx.x; i < n; i += kIT) pm[i] = i;
      __syncthreads();
      auto test = [&](const d4& v, int br, int bc) {
        const double e[4] = {v[0], v[1], v[2], v[3]};
        const int col = bc * 16 + li;
        double sv[4];
        int pp[4], qq[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = br * 16 + lk + 4 * r;
          const bool keep = row < n && col < n && row != col && !(br == bc && row > col);
          pp[r] = keep ? min(row, col) : -1;
          qq[r] = max(row, col);
          sv[r] = keep ? S[(int64_t)pp[r] * n + qq[r]] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (pp[r] < 0) continue;
          const double lp = dg[pp[r]], lq = dg[qq[r]], rr = -e[r];
          const double d = fabs(lq - lp);
          if (p.closec * fabs(sv[r] + lq * rr) >= d || p.closec * fabs(sv[r] + lp * rr) >= d) atomicMax(&pm[pp[r]], qq[r]);
        }
      };
#pragma unroll
      for (int j = 0; j < B::NC; ++j) test(acc[j], w, B::col(w, j));
      if (e_live) test(ace, kIBlk - 1, B::ce(w));
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kIT) {
        p.cl[it.e_off + i] = pm[i];
        p.lam_pre[it.e_off + i] = dg[i];
      }
    }
  }
}

// The work-group's items: sel[i] (or i without a list) for i = blockIdx.x,
// blockIdx.x + gridDim.x, ... below n_items.
template <class P>
__global__ __launch_bounds__(kIT, 1) void igemm_kernel(const ItemDev* __restrict__ items,
                                                       const int32_t* __restrict__ sel, int n_items, P p) {
  __shared__ double lds[2][2][kIPanelLds];
  __shared__ double dg[P::DIAG_A || P::DIAG_B || P::REACH ? kIN : 1];
  __shared__ int pm[P::PERM || P::REACH ? kIN : 1];
  if ((int)blockIdx.x >= n_items) return;
  typename Mat<typename P::TA>::raw_t ra[kIStage];
  typename Mat<typename P::TB>::raw_t rb[kIStage];
  {
    const int item = sel ? sel[blockIdx.x] : blockIdx.x;
    ifetch_pass<P, 0>(ra, rb, p, items[item], item, 0);
  }
  int buf = 0;
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int item = sel ? sel[i] : i;
    const ItemDev it = items[item];
    ipass<P, 0>(p, items, sel, n_items, i, item, it, lds, dg, pm, buf, ra, rb);
    ipass<P, 1>(p, items, sel, n_items, i, item, it, lds, dg, pm, buf, ra, rb);
  }
}

// Y = V X + H0 X
template <typename XT>
struct IgY {
  using TA = double;
  using TB = XT;
  static constexpr bool KA = true, KB = true, DIAG_A = true, DIAG_B = false, PERM = false, REACH = false;
  static constexpr int OUT = kOutF64, NPASS = 2;
  static constexpr int set(int ps) { return ps == 0 ? kSetLo : kSetHi; }
  static constexpr bool same_panel(int) { return false; }
  const GridDev* grids;
  const double* v64;
  const XT* xin;
  int xin_ws;
  double* work;
  __device__ const XT* X(const ItemDev& it) const {
    return xin_ws ? reinterpret_cast<const XT*>(WS(work, it).P1) : (xin + it.v_off);
  }
  // A = V + H0 (H0 added to the staged diagonal); V is symmetric: its rows
  // are read as the columns of A
  __device__ Mat<double> viewA(const ItemDev& it, int) const { return col_view(v64 + it.v_off, it.n, it.n); }
  __device__ double diag(const ItemDev& it, int i) const { return grids[it.grid].e0[i % it.N]; }
  template <int PS>
  __device__ Mat<XT> viewB(const ItemDev& it, int) const { return col_view(X(it), it.n, it.n); }
  template <int PS>
  __device__ __amdgpu_buffer_rsrc_t out(const ItemDev& it, int) const {
    return Mat<double>(WS(work, it).Y, (int64_t)it.n * it.n, 0, 0).r;
  }
  template <int PS>
  __device__ void store(const ItemDev&, int, bool, int, int, double) const {}
};
// S = X^T Y (pass 0) and G = X^T X (pass 1), symmetric
template <typename XT>
struct IgSG {
  using TA = XT;
  using TB = double;
  static constexpr bool KA = true, KB = true, DIAG_A = false, DIAG_B = false, PERM = false, REACH = true;
  static constexpr int OUT = kOutSym, NPASS = 2;
  static constexpr int set(int) { return kSetSym; }
  static constexpr bool same_panel(int ps) { return ps == 1; }
  const XT* xin;
  int xin_ws;
  double* work;
  double* lam_pre;  // close-pair test (refine_reach_kernel's outputs)
  int32_t* cl;
  double closec;
  __device__ Mat<XT> viewA(const ItemDev& it, int) const {
    const XT* X = xin_ws ? reinterpret_cast<const XT*>(WS(work, it).P1) : (xin + it.v_off);
    return col_view(X, it.n, it.n);
  }
  template <int PS>
  __device__ Mat<double> viewB(const ItemDev& it, int) const { return col_view<double>(WS(work, it).Y, it.n, it.n); }
  __device__ double diag(const ItemDev&, int) const { return 0.0; }
  template <int PS>
  __device__ __amdgpu_buffer_rsrc_t out(const ItemDev& it, int) const {
    const WS ws(work, it);
    return Mat<double>(PS == 0 ? ws.S : ws.G, (int64_t)it.n * it.n, 0, 0).r;
  }
  template <int PS>
  __device__ void store(const ItemDev&, int, bool, int, int, double) const {}
};
// X' = X M (M in W6)
template <typename XT>
struct IgXM {
  using TA = XT;
  using TB = double;
  static constexpr bool KA = false, KB = true, DIAG_A = false, DIAG_B = false, PERM = true, REACH = false;
  static constexpr int OUT = kOutF64, NPASS = 2;
  static constexpr int set(int ps) { return ps == 0 ? kSetLo : kSetHi; }
  static constexpr bool same_panel(int) { return false; }
  const XT* xin;
  int xin_ws;
  double* evec;
  int xout_ws;
  double* work;
  const int32_t* perm;  // column c of the result goes to column perm[e_off + c] (or nullptr)
  __device__ Mat<XT> viewA(const ItemDev& it, int) const {
    const XT* X = xin_ws ? reinterpret_cast<const XT*>(WS(work, it).P1) : (xin + it.v_off);
    return row_view(X, it.n, it.n);
  }
  template <int PS>
  __device__ Mat<double> viewB(const ItemDev& it, int) const { return col_view<double>(WS(work, it).W6, it.n, it.n); }
  __device__ double diag(const ItemDev&, int) const { return 0.0; }
  template <int PS>
  __device__ __amdgpu_buffer_rsrc_t out(const ItemDev& it, int) const {
    return Mat<double>(xout_ws ? WS(work, it).P1 : (evec + it.v_off), (int64_t)it.n * it.n, 0, 0).r;
  }
  template <int PS>
  __device__ void store(const ItemDev&, int, bool, int, int, double) const {}
};

// Warm start of the LDS Jacobi: Z = Q0^T H for a warm item (Q0: its
// reference's eigenvectors, column-major floats at the reference's
// work-space), i.e. Z[i][j] = (H Q0)[j][i], stored as floats row-major =
// H Q0 column-major in the item's x32.  The FP64 matrix cores take V + H0
// (H0 added to the staged diagonal of B).
struct IgWarm {
  using TA = float;
  using TB = double;
  static constexpr bool KA = false, KB = true, DIAG_A = false, DIAG_B = true, PERM = false, REACH = false;
  static constexpr int OUT = kOutF32, NPASS = 2;
  static constexpr int set(int ps) { return ps == 0 ? kSetLo : kSetHi; }
  static constexpr bool same_panel(int) { return false; }
  const ItemDev* items;
  const int32_t* ref;
  const GridDev* grids;
  const double* v64;
  float* x32;
  const double* work;
  __device__ const float* Q0(int item) const { return reinterpret_cast<const float*>(work + items[ref[item]].w_off); }
  // A(i, k) = Q0[i n + k] (row i of A = column i of Q0)
  __device__ Mat<float> viewA(const ItemDev& it, int item) const { return row_view(Q0(item), it.n, it.n); }
  template <int PS>
  __device__ Mat<double> viewB(const ItemDev& it, int) const { return col_view(v64 + it.v_off, it.n, it.n); }
  __device__ double diag(const ItemDev& it, int i) const { return grids[it.grid].e0[i % it.N]; }
  template <int PS>
  __device__ __amdgpu_buffer_rsrc_t out(const ItemDev& it, int) const {
    return Mat<float>(x32 + it.v_off, (int64_t)it.n * it.n, 0, 0).r;
  }
  template <int PS>
  __device__ void store(const ItemDev&, int, bool, int, int, double) const {}
};

}  // namespace

hipError_t launch_refine(const ItemDev* items, int n_items, int min_n, int max_n, const GridDev* grids,
                         const double* v64, const float* x32, double* evec, double* eval, double* lam_pre,
                         double* work, int32_t* cl, int32_t* status, int steps, int close_log10, int gemm,
                         int rr_steps, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  if (max_n > kMaxN) return hipErrorInvalidValue;
  const int nt = (max_n + kTM - 1) / kTM;  // 64-row blocks of form_m
  const int nt2 = (max_n + T64::TM - 1) / T64::TM;  // GEMM tiles
  const int tiles = nt2 * nt2, up_tiles = nt2 * (nt2 + 1) / 2;
  // whole-item products when every item has 193..208 rows (unless tiles are asked for)
  const bool whole = gemm == 0 && min_n >= kINMin && max_n <= kIN;
  unsigned ig = 0;  // persistent grid: one work-group per CU
  if (whole) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    ig = (unsigned)(n_items < cus ? n_items : cus);
  }
  int cur_ws = 0;  // X in the caller's evec (0) or in the work-space P1 (1); step 0 reads x32
  for (int st = 0; st < steps; ++st) {
    // whole-item products: the last step's X M goes to evec already sorted
    // (refine_rank_kernel), the earlier ones alternate so that it reads P1
    const bool last = st == steps - 1;
    const int out_ws = whole ? ((steps - 1 - st) % 2 == 0 ? 0 : 1) : (st == 0 ? 0 : 1 - cur_ws);
    double closec = 1.0;
    for (int q = 0; q < close_log10 + 2 * st; ++q) closec *= 10.0;
    if (whole) {
      if (st == 0) {
        hipLaunchKernelGGL(igemm_kernel<IgY<float>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgY<float>{grids, v64, x32, 0, work});
        hipLaunchKernelGGL(igemm_kernel<IgSG<float>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgSG<float>{x32, 0, work, lam_pre, cl, closec});
      } else {
        hipLaunchKernelGGL(igemm_kernel<IgY<double>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgY<double>{grids, v64, (const double*)evec, cur_ws, work});
        hipLaunchKernelGGL(igemm_kernel<IgSG<double>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgSG<double>{(const double*)evec, cur_ws, work, lam_pre, cl, closec});
      }
    } else if (st == 0) {
      hipLaunchKernelGGL(gemm_y_kernel<float>, dim3(xcd_grid(tiles, n_items)), dim3(T64::NT), 0, s, items, n_items,
                         grids, v64, x32, 0, work, tiles);
      hipLaunchKernelGGL(gemm_sg_kernel<float>, dim3(xcd_grid(up_tiles, n_items)), dim3(T64::NT), 0, s, items,
                         n_items, x32, 0, work, up_tiles);
    } else {
      hipLaunchKernelGGL(gemm_y_kernel<double>, dim3(xcd_grid(tiles, n_items)), dim3(T64::NT), 0, s, items, n_items,
                         grids, v64, (const double*)evec, cur_ws, work, tiles);
      hipLaunchKernelGGL(gemm_sg_kernel<double>, dim3(xcd_grid(up_tiles, n_items)), dim3(T64::NT), 0, s, items,
                         n_items, (const double*)evec, cur_ws, work, up_tiles);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (!whole) {  // the whole-item S, G product ran the close-pair test itself
      const int rt = (max_n + kReachRows - 1) / kReachRows;
      hipLaunchKernelGGL(refine_reach_kernel, dim3(xcd_grid(rt, n_items)), dim3(64 * kReachWaves), 0, s, items,
                         lam_pre, work, cl, closec, rt, n_items);
    }
    // a step without Rayleigh-Ritz: M = I + E for every column (close pairs
    // take R_ij/2), no chain kernel
    const bool rr = rr_steps <= 0 || st >= steps - rr_steps;
    if (!rr) {
      hipLaunchKernelGGL(form_m_kernel, dim3(xcd_grid(form_m_tiles(max_n), n_items)), dim3(kBlock), 0, s, items,
                         lam_pre, work, (const int32_t*)nullptr, closec, form_m_tiles(max_n), n_items);
    }
    // M: the columns outside chains (form_m, streaming S and G) on the side
    // stream while the chain kernel (latency-bound) writes the chain columns
    hipStream_t sm = s;
    if (rr && side != nullptr) {
      err = hipEventRecord(fork, s);
      if (err == hipSuccess) err = hipStreamWaitEvent(side, fork, 0);
      if (err != hipSuccess) return err;
      sm = side;
    }
    if (rr)
      hipLaunchKernelGGL(form_m_kernel, dim3(xcd_grid(form_m_tiles(max_n), n_items)), dim3(kBlock), 0, sm, items,
                         lam_pre, work, cl, closec, form_m_tiles(max_n), n_items);
    // Rayleigh-Ritz of the chains to FP64 accuracy in the last step; in an
    // earlier one the Newton columns keep second-order errors of up to
    // 1/c^2 = 1e-6 and the next step squares what is left, so the chains'
    // Jacobi stops after a sweep whose largest rotation was below 1e-6 (the
    // cosines left are then of order 1e-12)
    if (rr) {
      hipLaunchKernelGGL(refine_chain_kernel, dim3(n_items), dim3(kBlock), 0, s, items, lam_pre, eval, work, cl,
                         status, closec, last ? 1e-15 : 1e-12, last ? 8e-15 : 1e-6);
      if (max_n > kMaxChain) {
        err = hipFuncSetAttribute(reinterpret_cast<const void*>(refine_bigchain_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kBigDynDoubles * sizeof(double)));
        if (err != hipSuccess) return err;
      }
      if (max_n > kMaxChain)
        hipLaunchKernelGGL(refine_bigchain_kernel, dim3(n_items), dim3(kBlock), kBigDynDoubles * sizeof(double), s,
                           items, lam_pre, eval, work, status, closec, last ? 1e-15 : 1e-12, last ? 8e-15 : 1e-6);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (rr && side != nullptr) {
      err = hipEventRecord(join, side);
      if (err == hipSuccess) err = hipStreamWaitEvent(s, join, 0);
      if (err != hipSuccess) return err;
    }
    if (whole && last)
      hipLaunchKernelGGL(refine_rank_kernel, dim3(n_items), dim3(kBlock), 0, s, items, eval, cl, status);
    if (whole) {
      if (st == 0)
        hipLaunchKernelGGL(igemm_kernel<IgXM<float>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgXM<float>{x32, 0, evec, out_ws, work, last ? cl : nullptr});
      else
        hipLaunchKernelGGL(igemm_kernel<IgXM<double>>, dim3(ig), dim3(kIT), 0, s, items, nullptr, n_items,
                           IgXM<double>{(const double*)evec, cur_ws, evec, out_ws, work, last ? cl : nullptr});
    } else if (st == 0)
      hipLaunchKernelGGL(gemm_xm_kernel<float>, dim3(xcd_grid(tiles, n_items)), dim3(T64::NT), 0, s, items, n_items,
                         x32, 0, evec, out_ws, work, tiles);
    else
      hipLaunchKernelGGL(gemm_xm_kernel<double>, dim3(xcd_grid(tiles, n_items)), dim3(T64::NT), 0, s, items, n_items,
                         (const double*)evec, cur_ws, evec, out_ws, work, tiles);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    cur_ws = out_ws;
  }
  if (!whole)
    hipLaunchKernelGGL(refine_finish_kernel, dim3(n_items), dim3(kBlock), 0, s, items, evec, cur_ws, work, eval,
                       status);
  return hipGetLastError();
}

}  // namespace wpcd

namespace wpcd {

hipError_t launch_rayleigh_f64(const ItemDev* items, int n_items, int max_n, const GridDev* grids,
                               const double* v64, double* work, double* evec, double* eval, int32_t* status,
                               hipStream_t s) {
  if (max_n > kMaxN) return hipErrorInvalidValue;
  const int nt = (max_n + T64::TM - 1) / T64::TM;
  hipLaunchKernelGGL(rq_hx_kernel, dim3(xcd_grid(nt * nt, n_items)), dim3(T64::NT), 0, s, items, n_items, grids, v64,
                     work, nt * nt);
  hipLaunchKernelGGL(rq_sort_kernel, dim3(n_items), dim3(kBlock), 0, s, items, work, evec, eval, status);
  return hipGetLastError();
}

}  // namespace wpcd

namespace wpcd {

hipError_t launch_warm_pick(const ItemDev* items, int n_items, const int32_t* jlist, const int32_t* pick, int n_pick,
                            const int32_t* cand, float* sig, const double* v64, int32_t* ref, hipStream_t s) {
  if (n_pick == 0) return hipSuccess;
  hipLaunchKernelGGL(warm_sig_kernel, dim3(n_items), dim3(kBlock), 0, s, items, v64, sig);
  hipLaunchKernelGGL(warm_pick_kernel, dim3(n_pick), dim3(kBlock), 0, s, pick, jlist, cand, (const float*)sig, ref);
  return hipGetLastError();
}

hipError_t launch_jacobi_warm_prep(const ItemDev* items, int n_items, const int32_t* refs, int n_refs,
                                   const int32_t* warm, int n_warm, int32_t* ref, int min_n, int max_n,
                                   const int32_t* jlist, const int32_t* pick, int n_pick, const int32_t* cand,
                                   float* sig, const GridDev* grids, const double* v64, float* x32, double* work,
                                   hipStream_t s) {
  if (max_n > kMaxN) return hipErrorInvalidValue;
  if (n_refs == 0 || n_warm == 0) return hipSuccess;
  if (n_pick > 0) {
    hipError_t e = launch_warm_pick(items, n_items, jlist, pick, n_pick, cand, sig, v64, ref, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(warm_q0_kernel, dim3(n_refs), dim3(kBlock), 0, s, items, refs, x32, work);
  if (min_n >= kINMin && max_n <= kIN) {  // whole-item products, one work-group per CU
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(igemm_kernel<IgWarm>, dim3(n_warm < cus ? n_warm : cus), dim3(kIT), 0, s, items, warm, n_warm,
                       IgWarm{items, ref, grids, v64, x32, work});
    return hipGetLastError();
  }
  const int nt = (max_n + T64::TM - 1) / T64::TM;
  hipLaunchKernelGGL(warm_y_kernel, dim3(xcd_grid(nt * nt, n_warm)), dim3(T64::NT), 0, s, items, warm, n_warm, ref,
                     grids, v64, x32, work, nt * nt);
  return hipGetLastError();
}

}  // namespace wpcd
