// Host-side handle types of the C ABI (shared by the library's host sources).
#pragma once

#include <string>
#include <vector>

#include "internal.h"

namespace wpcd {

struct GridHost {
  int N = 0, ng = 0;
  std::vector<double> kb, nodes, weights;
  double* dbuf = nullptr;
  GridDev dev{};
};

// Records msg as this thread's wpcd_last_error() text; returns code.
int set_error(int code, const char* msg);

struct BasisHost {
  int grid = 0, nch = 0, n = 0, n_terms = 0;
  double* dbuf = nullptr;  // n_terms * n * n FP64
};

}  // namespace wpcd


struct wpcd_context {
  int device = 0;
  wpcd_config cfg{};
  std::vector<wpcd::GridHost> grids;
  std::vector<wpcd::BasisHost> bases;
  // stage timers
  bool profiling = false;
  struct Pending {
    int stage;
    hipEvent_t start, stop;
  };
  std::vector<Pending> pending;
  double stage_ms[WPCD_N_STAGES] = {0};
  int64_t stage_launches[WPCD_N_STAGES] = {0};
  unsigned long long* d_counters = nullptr;  // LDS Jacobi work counters (while profiling)
  // second stream of the refinement (default priority) and its fork/join events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // first failed HIP call of a compute call (then every compute call returns
  // WPCD_ERR_DEVICE)
  bool sticky = false;
  std::string sticky_msg;
};

struct wpcd_batch_s {
  wpcd_ctx ctx = nullptr;
  int device = 0;  // the context's device (destroy must not read the context: it may be gone)
  int n_items = 0, n_samples = 0, max_n = 0, min_n = 0, max_nbins = 0;
  int warm_min_n = 0, warm_max_n = 0;  // sizes of the warm-started items
  std::vector<wpcd::ItemDev> h_items;
  wpcd::ItemDev* d_items = nullptr;
  wpcd::GridDev* d_grids = nullptr;
  int32_t* d_sample_ptr = nullptr;
  int32_t* d_sample_items = nullptr;
  wpcd::BasisDev* d_bases = nullptr;
  int n_fine = 0, n_affine = 0;  // items projected from u_fine / from a basis
  int64_t u_elems = 0, v_elems = 0, eval_elems = 0, t_doubles = 0, delta_elems = 0, mix_elems = 0, work_doubles = 0,
          coef_elems = 0;
  float* d_x32 = nullptr;
  double* d_work = nullptr;
  int32_t* d_cl = nullptr;
  double* d_lam = nullptr;  // Rayleigh quotients of the current refinement step
  // items grouped by eigensolver size class (wpcd::size_class); class c holds
  // d_class[class_ptr[c] .. class_ptr[c+1]) with largest n class_maxn[c]
  int32_t* d_class = nullptr;
  int class_ptr[wpcd::kNumClasses + 1] = {0};
  int class_maxn[wpcd::kNumClasses] = {0};
  // warm start of the FP32 Jacobi (wpcd_config.jacobi_start): d_jlist holds
  // the segments cold_0 .. cold_{C-1}, warm_0 .. warm_{C-1}, refs (C size
  // classes), segment t at [jl_ptr[t], jl_ptr[t + 1]); the warm segments are
  // contiguous; d_ref gives each warm item its reference (-1 otherwise)
  static constexpr int kC = wpcd::kNumClasses;
  int32_t* d_jlist = nullptr;
  int32_t* d_ref = nullptr;
  int jl_ptr[2 * kC + 2] = {0};
  // reference choice of the LDS-class warm items (on the device, from a
  // strided sample of V): d_cand holds each group's cold items, d_pick one
  // task per run of up to 16 warm items of one group (jlist offset, count,
  // candidate offset, count), d_sig the samples (kWarmSig floats per item)
  int32_t* d_cand = nullptr;
  int32_t* d_pick = nullptr;
  float* d_sig = nullptr;
  int n_pick = 0;
  // convergence feedback and launch counters of the device-memory Jacobi
  wpcd::JacFeedback jfb;
};

struct wpcd_mi_s {
  wpcd_ctx ctx = nullptr;
  int device = 0;  // the context's device (destroy must not read the context: it may be gone)
  int n_items = 0, n_samples = 0, nq = 0, ne = 0, max_nch = 0;
  double cutoff = 0.0;
  std::vector<wpcd::MiItemDev> h_items;
  std::vector<double> pts, wts;  // N_Q nodes then the N_E on-shell momenta; N_Q weights
  int64_t u_elems = 0, k_elems = 0, d_elems = 0, m_elems = 0;
  wpcd::MiItemDev* d_items = nullptr;
  double* d_pts = nullptr;   // N_Q + N_E points
  double* d_qw = nullptr;    // N_Q weights
  double* d_loss = nullptr;  // per (item, energy): (2J+1) sum_a (1 - Re S_aa)
  int32_t* d_sample_ptr = nullptr;
  int32_t* d_sample_items = nullptr;
};
