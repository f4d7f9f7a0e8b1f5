// Internal declarations of the WPCD HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "wpcd.h"

namespace wpcd {

// Device view of a resident bin grid.
// Momentum packets (f = 1, N_i = dk_i) and energy packets (f = sqrt(2k),
// N_i = dE_i) differ only in these tables.
struct GridDev {
  const double* kb;    // N+1 bin boundaries k_j
  const double* eb;    // N+1 boundary energies k_j^2
  const double* dk;    // N: N_i/f(q_i)^2 (the bin width for momentum packets)
  const double* kbar;  // N on-shell momenta q_i (the bin midpoints for momentum packets)
  const double* e0;    // N free-Hamiltonian diagonal <x_i|k^2|x_i>
  const double* wk;    // N*ng Gauss weight times node times f(node), bin-major
  const double* rsdk;  // N 1/sqrt(N_i)
  int32_t N;
  int32_t ng;
};

// Device descriptor of one item of a batch.
struct ItemDev {
  int32_t grid;    // index into the grid table
  int32_t nch;     // 1 or 2
  int32_t N;       // bins
  int32_t n;       // nch*N
  int32_t ng;      // Gauss nodes per bin
  int32_t J;
  int32_t sample;
  int32_t basis;   // -1: fine-mesh potential; >= 0: index into the basis table
  int32_t spin;    // total spin S (0 or 1), -1 if not given
  int32_t l0;      // orbital l of the first channel (J - 1 for coupled items), -1 if not given
  int64_t u_off;   // elements into u_fine
  int64_t v_off;   // elements into v64 / evec (n*n)
  int64_t e_off;   // elements into eval (n)
  int64_t t_off;   // doubles into t (2*N*nch*nch)
  int64_t d_off;   // elements into delta / s_dev (N*nch)
  int64_t m_off;   // elements into mix (N)
  int64_t w_off;   // elements into the per-item eigensolver workspace
  int64_t c_off;   // elements into the affine coefficient array
};

// Device view of a resident projected basis: n_terms consecutive n*n FP64
// matrices B_t (row-major, exactly symmetric).
struct BasisDev {
  const double* b;
  int32_t n;
  int32_t n_terms;
};

// Largest matrix the FP32 LDS eigensolver holds (n*n floats must fit 160 KiB).
constexpr int kMaxLdsN = 200;
// Size classes of the eigensolver launches: n <= 64, <= 128, <= 200 (LDS) and
// larger (device memory).
constexpr int kNumClasses = 4;
inline int size_class(int n) { return n <= 64 ? 0 : (n <= 128 ? 1 : (n <= kMaxLdsN ? 2 : 3)); }
// Largest item the library accepts.
constexpr int kMaxN = 1200;

// Kernel launchers (each returns hipSuccess or the launch error).
// generic: some fine-mesh item is not taken by the tiled kernel (project_tiled)
hipError_t launch_project(const ItemDev* items, int n_items, int max_n, const GridDev* grids, const void* u,
                          int u_dtype, double* v64, bool generic, hipStream_t s);
// fine-mesh items projected by the tiled ng = 8 kernel: their U block starts
// on a 16-byte boundary (u: the caller's U buffer, elem: its element size)
__host__ __device__ inline bool project_tiled(const ItemDev& it, const void* u, int elem) {
  return it.ng == 8 && (((uintptr_t)u + (uintptr_t)it.u_off * (uintptr_t)elem) & 15) == 0;
}
hipError_t launch_project_affine(const ItemDev* items, int n_items, int max_n, const BasisDev* bases,
                                 const double* coef, double* v64, hipStream_t s);
hipError_t launch_jacobi_f32_lds(const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                 const GridDev* grids, const double* v64, float* x32, double* eval,
                                 int32_t* status, int max_sweeps, float tol, float stop, int block_cols,
                                 const int32_t* ref, const double* work, unsigned long long* counters,
                                 hipStream_t s);
// Warm start of the LDS Jacobi (items with a reference, ref[item] >= 0):
// writes each reference's eigenvectors, columns in descending eigenvalue
// order, column-major as floats into the reference's work-space, then
// H Q0 of every warm item, column-major FP32, into the item's x32 (min_n,
// max_n: the warm items' smallest and largest n).  Before that, each pick
// task (jlist offset, count, candidate offset, count; n_pick of them) sets
// ref[] of up to kWarmPick warm items of one group to the candidate whose V
// is nearest to theirs on a strided sample of kWarmSig entries (sig: kWarmSig
// floats per item of the batch, n_items of them).
constexpr int kWarmPick = 16;
constexpr int kWarmSig = 1024;
// The reference choice alone (it needs V only, not the cold solutions): the
// caller may run it beside the cold Jacobi and pass n_pick = 0 below.
hipError_t launch_warm_pick(const ItemDev* items, int n_items, const int32_t* jlist, const int32_t* pick, int n_pick,
                            const int32_t* cand, float* sig, const double* v64, int32_t* ref, hipStream_t s);
hipError_t launch_jacobi_warm_prep(const ItemDev* items, int n_items, const int32_t* refs, int n_refs,
                                   const int32_t* warm, int n_warm, int32_t* ref, int min_n, int max_n,
                                   const int32_t* jlist, const int32_t* pick, int n_pick, const int32_t* cand,
                                   float* sig, const GridDev* grids, const double* v64, float* x32, double* work,
                                   hipStream_t s);
// Convergence feedback of the device-memory Jacobi.  With it (and a stream
// that is not being captured) the sweeps are enqueued a few at a time: after
// each sweep a one-work-group kernel writes 1 into flag[sweep] (pinned host
// memory, written by the device) when every item of the launch has
// converged, and the host, kJacLookahead sweeps behind the device, stops
// enqueueing once a flag it has waited for is set.  Without it every sweep
// up to max_sweeps is enqueued (converged items return at once); a feedback
// object without flags only counts.  One feedback object serves one launch
// sequence at a time.
constexpr int kJacFbEvents = 4;
constexpr int kJacLookahead = 2;
struct JacFeedback {
  int32_t* flag = nullptr;  // 64 ints, hipHostMalloc'd; the device writes them
  hipEvent_t ev[kJacFbEvents] = {};
  int64_t launches = 0;     // kernel launches of the device-memory Jacobi since the counters were cleared
  int64_t sweeps = 0;       // sweeps enqueued since the counters were cleared
};
hipError_t jac_feedback_create(JacFeedback& f);
void jac_feedback_destroy(JacFeedback& f);
hipError_t launch_jacobi_global(int mixed, const ItemDev* items, const int32_t* sel, int n_sel, int max_n,
                                const GridDev* grids, const double* v64, double* work, double* evec, float* x32,
                                double* eval, int32_t* status, int max_sweeps, double tol, double stop,
                                const int32_t* ref, JacFeedback* fb, hipStream_t s);
// FP64 device-memory Jacobi epilogue: Rayleigh quotients x^T H x of the
// normalised columns it left in the work-space (MFMA product H X), sort by
// them, write eval and the row-major evec of every item of the batch.
hipError_t launch_rayleigh_f64(const ItemDev* items, int n_items, int max_n, const GridDev* grids,
                               const double* v64, double* work, double* evec, double* eval, int32_t* status,
                               hipStream_t s);
// gemm: 0 = whole-item products when every item has 193..208 rows, else
// 64 x 64 tiles; 1 = tiles.  rr_steps: the last rr_steps steps solve
// clusters by Rayleigh-Ritz (0 = all).  side (with two events, or nullptr):
// a second stream on which part of each step runs concurrently; the work on
// s waits for it before going on.
hipError_t launch_refine(const ItemDev* items, int n_items, int min_n, int max_n, const GridDev* grids,
                         const double* v64, const float* x32, double* evec, double* eval, double* lam_pre,
                         double* work, int32_t* cl, int32_t* status, int steps, int close_log10, int gemm,
                         int rr_steps, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join);
hipError_t launch_tmatrix(const ItemDev* items, int n_items, int max_n, const GridDev* grids, const double* v64,
                          const double* eval, const double* evec, int mode, double* t, int32_t* status,
                          hipStream_t s);
hipError_t launch_observables(const ItemDev* items, int n_items, int max_nbins, const GridDev* grids,
                              const double* t, double* delta, double* mix, double* s_dev, hipStream_t s);
hipError_t launch_saclay(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                         int n_samples, const GridDev* grids, const double* delta, const double* mix,
                         const double* tlab, int n_tlab, const double* theta_deg, int n_theta, double* amp,
                         double* dsdo, hipStream_t s);
hipError_t launch_sigma(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                        int n_samples, const GridDev* grids, const double* delta, const double* mix,
                        const double* tlab, const int32_t* tlab_off, int n_tlab, double* sigma, hipStream_t s);
hipError_t launch_sigma_band(const ItemDev* items, const int32_t* sample_ptr, const int32_t* sample_items,
                             int n_samples, const GridDev* grids, const double* delta, const double* mix,
                             const double* tlab, int n_tlab, const double* fracs, int n_frac, double* sigma_lo,
                             double* sigma_hi, hipStream_t s);

// Matrix-inversion solver (the paper's comparison method): one item = one
// channel of one sample, solved at every energy of the solver object.
struct MiItemDev {
  int32_t nch;     // 1 or 2
  int32_t J;
  int32_t sample;
  int32_t pad;
  int64_t u_off;   // elements into u: (nch (N_Q + N_E))^2, channel-major
  int64_t k_off;   // elements into kmat: N_E nch^2
  int64_t d_off;   // elements into delta: N_E nch
  int64_t m_off;   // elements into mix: N_E
};
// Largest quadrature mesh of the MI solver (the augmented FP64 system of an
// uncoupled item, 141 x 142 doubles, fills the LDS; coupled items: 69).
constexpr int kMaxMiNq = 140;
size_t mi_lds_bytes(int nq, int K);
hipError_t launch_mi_solve(const MiItemDev* items, int n_items, int nq, int ne, int max_nch, const double* qw,
                           const double* pts, double cutoff, const double* u, double* kmat, double* delta,
                           double* mix, double* loss, const int32_t* sample_ptr, const int32_t* sample_items,
                           int n_samples, double* sigma, int32_t* status, hipStream_t s);

// Per-item device work-space (doubles) of the eigensolvers for an n x n item:
// P1 | Y | S | G | W5 | W6 | W7 for the refinement; the device-memory Jacobi
// keeps W (n*n elements) and its per-item state (<= 320 bytes) at the start.
inline int64_t eig_work_doubles(int n) { return 7LL * n * n + 40; }

}  // namespace wpcd
