// Host side of the C ABI: contexts, resident grids, batches and the compute
// entry points declared in include/wpcd.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "handles.h"
#include "internal.h"

using namespace wpcd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? WPCD_ERR_NOMEM : WPCD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define WPCD_HIP(call, what)              \
  do {                                    \
    hipError_t e_ = (call);               \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// A failed HIP call inside a compute call leaves the context's device state
// unknown: the first such failure is recorded, and every later compute call
// on the context returns WPCD_ERR_DEVICE with its message (allocation
// failures are not recorded: they leave nothing half done).
int dev_fail(wpcd_ctx ctx, hipError_t e, const char* what) {
  const int code = hip_fail(e, what);
  if (code == WPCD_ERR_DEVICE && !ctx->sticky) {
    ctx->sticky = true;
    ctx->sticky_msg = g_err;
  }
  return code;
}

#define WPCD_HIPX(ctx, call, what)                       \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return dev_fail(ctx, e_, what); \
  } while (0)

// Entry check of the compute calls: a recorded device failure is sticky.
#define WPCD_STICKY(ctx)                                                                                  \
  do {                                                                                                    \
    if ((ctx)->sticky)                                                                                    \
      return fail(WPCD_ERR_DEVICE, "an earlier call failed on the device: %s", (ctx)->sticky_msg.c_str()); \
  } while (0)

// Runs `launch` (returning hipError_t) between two events on `stream` when the
// context's stage timers are on.
template <class F>
hipError_t timed(wpcd_ctx ctx, int stage, hipStream_t stream, F launch) {
  if (!ctx->profiling) return launch();
  wpcd_context::Pending p{stage, nullptr, nullptr};
  hipError_t e = hipEventCreate(&p.start);
  if (e == hipSuccess) e = hipEventCreate(&p.stop);
  if (e == hipSuccess) e = hipEventRecord(p.start, stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(p.stop, stream);
  if (e == hipSuccess) {
    ctx->pending.push_back(p);
  } else {
    if (p.start) hipEventDestroy(p.start);
    if (p.stop) hipEventDestroy(p.stop);
  }
  return e;
}

// Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n, with
// P_n'(x) = n (x P_n - P_{n-1})/(x^2 - 1) and w = 2/((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int iter = 0; iter < 100; ++iter) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) <= 1e-16) {
        // derivative at the converged root
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[n - 1 - i] = z;  // ascending
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

namespace wpcd {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace wpcd

// ------------------------------------------------ static eigensolver scratch
// The eigensolver work-space of wpcd_eigh_noalloc lives in this file-scope
// device array (one copy per device, held until the process ends) instead of
// the batch's own allocation.  In host code `scratch` only names the symbol:
// its device address on the current device comes from hipGetSymbolAddress,
// looked up once per device (at the first wpcd_eigh_noalloc call there, with
// the device current) and kept in g_scratch; kernels only ever receive that
// address.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// With `dev` current: the device address of `scratch` on it (nullptr if the
// lookup failed; the next call tries again, and the failure is cleared from
// HIP's last-error state so that no later launch check reports it).
unsigned char* scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    if (e == hipSuccess && p) g_scratch[dev] = static_cast<unsigned char*>(p);
    else (void)hipGetLastError();
  }
  return g_scratch[dev];
}

unsigned char* scratch_ptr(int dev) { return scratch_lookup(dev); }

const char* scratch_error(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return "device index beyond the scratch table";
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_err[dev] == hipSuccess ? "scratch address unavailable" : hipGetErrorString(g_scratch_err[dev]);
}

// Byte offsets of the work-space arrays of a batch inside the scratch, each
// on a 256-byte boundary.
struct ScratchPlan {
  size_t x32, work, cl, lam, sig, total;
};
ScratchPlan scratch_plan(const wpcd_batch_s* b) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  ScratchPlan p{};
  size_t o = 0;
  p.x32 = o;
  o = up(o + sizeof(float) * (size_t)b->v_elems);
  p.work = o;
  o = up(o + sizeof(double) * (size_t)b->work_doubles);
  p.cl = o;
  o = up(o + sizeof(int32_t) * (size_t)b->eval_elems);
  p.lam = o;
  o = up(o + sizeof(double) * (size_t)b->eval_elems);
  p.sig = o;
  o = up(o + (b->n_pick > 0 ? sizeof(float) * kWarmSig * (size_t)b->n_items : 0));
  p.total = o;
  return p;
}

}  // namespace

extern "C" {

const char* wpcd_last_error(void) { return g_err.c_str(); }
const char* wpcd_version(void) { return "wpcd-gfx950 0.1"; }

int wpcd_create(wpcd_ctx* out, int hip_device, const wpcd_config* cfg) {
  if (!out) return fail(WPCD_ERR_INVALID, "wpcd_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  WPCD_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= ndev)
    return fail(WPCD_ERR_INVALID, "wpcd_create: device %d out of range (%d devices)", hip_device, ndev);
  wpcd_config c{30, 2, 2e-7, 1e-15, 0, 0, 0.0, 0, 0, 0};
  if (cfg) c = *cfg;
  if (c.refine_close_log10 == 0) c.refine_close_log10 = 3;
  // default stop 1e-4: rotations up to that size left in the FP32 vectors are
  // taken by the FP64 refinement (quadratic: about 1e-8 after its first step)
  // without growing its chains; 3e-4 does grow them (coupled n = 200 batch:
  // 2.90 sweeps at 3e-5, 2.50 at 1e-4 with the same refinement time); never
  // below 8 x tol, where rotations at the skip threshold would recur
  if (c.jacobi_stop_f32 == 0.0) c.jacobi_stop_f32 = std::max(2e-4, 8.0 * c.jacobi_tol_f32);
  if (c.max_sweeps < 1 || c.max_sweeps > 60) return fail(WPCD_ERR_INVALID, "max_sweeps must be in [1, 60]");
  if (c.refine_steps < 0 || c.refine_steps > 4) return fail(WPCD_ERR_INVALID, "refine_steps must be in [0, 4]");
  if (!(c.jacobi_tol_f32 > 0) || !(c.jacobi_tol_f64 > 0)) return fail(WPCD_ERR_INVALID, "tolerances must be > 0");
  if (!(c.jacobi_stop_f32 > 0) || !(c.jacobi_stop_f32 < 1))
    return fail(WPCD_ERR_INVALID, "jacobi_stop_f32 must be in (0, 1) (0 = default)");
  if (c.jacobi_start != 0 && c.jacobi_start != 1) return fail(WPCD_ERR_INVALID, "jacobi_start must be 0 or 1");
  if (c.refine_gemm != 0 && c.refine_gemm != 1) return fail(WPCD_ERR_INVALID, "refine_gemm must be 0 or 1");
  if (c.jacobi_block < 0 || c.jacobi_block > 7)
    return fail(WPCD_ERR_INVALID, "jacobi_block must be in [0, 7]");
  if (c.refine_close_log10 < 1 || c.refine_close_log10 > 8)
    return fail(WPCD_ERR_INVALID, "refine_close_log10 must be in [1, 8] (0 = default)");
  if (c.refine_rr_steps < 0 || c.refine_rr_steps > 4)
    return fail(WPCD_ERR_INVALID, "refine_rr_steps must be in [0, 4] (0 = every step)");
  WPCD_HIP(hipSetDevice(hip_device), "hipSetDevice");
  wpcd_context* ctx = new (std::nothrow) wpcd_context;
  if (!ctx) return fail(WPCD_ERR_NOMEM, "wpcd_create: host allocation");
  ctx->device = hip_device;
  ctx->cfg = c;
  hipError_t e = hipMalloc((void**)&ctx->d_counters, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(ctx->d_counters, 0, 4 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    wpcd_destroy(ctx);
    return hip_fail(e, "wpcd_create: counters");
  }
  *out = ctx;
  return WPCD_OK;
}

void wpcd_destroy(wpcd_ctx ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  for (auto& p : ctx->pending) {
    hipEventSynchronize(p.stop);
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  for (auto& g : ctx->grids) hipFree(g.dbuf);
  for (auto& bs : ctx->bases) hipFree(bs.dbuf);
  hipFree(ctx->d_counters);
  if (ctx->side) {
    hipStreamSynchronize(ctx->side);
    hipStreamDestroy(ctx->side);
  }
  if (ctx->fork) hipEventDestroy(ctx->fork);
  if (ctx->join) hipEventDestroy(ctx->join);
  delete ctx;
}

int wpcd_grid_create(wpcd_ctx ctx, const double* k_bounds_host, int n_wp, int n_gauss, int* grid_id) {
  return wpcd_grid_create_packets(ctx, k_bounds_host, n_wp, n_gauss, WPCD_PACKET_MOMENTUM, grid_id);
}

int wpcd_grid_create_packets(wpcd_ctx ctx, const double* k_bounds_host, int n_wp, int n_gauss, int packet,
                             int* grid_id) {
  if (!ctx || !k_bounds_host || !grid_id) return fail(WPCD_ERR_INVALID, "wpcd_grid_create: NULL argument");
  if (packet != WPCD_PACKET_MOMENTUM && packet != WPCD_PACKET_ENERGY)
    return fail(WPCD_ERR_INVALID, "wpcd_grid_create: unknown packet kind %d", packet);
  if (n_wp < 2 || n_wp > kMaxN) return fail(WPCD_ERR_INVALID, "n_wp must be in [2, %d]", kMaxN);
  if (n_gauss < 1 || n_gauss > 16) return fail(WPCD_ERR_INVALID, "n_gauss must be in [1, 16]");
  if (k_bounds_host[0] != 0.0) return fail(WPCD_ERR_INVALID, "k_bounds[0] must be 0");
  for (int i = 1; i <= n_wp; ++i)
    if (!(k_bounds_host[i] > k_bounds_host[i - 1]) || !isfinite(k_bounds_host[i]))
      return fail(WPCD_ERR_INVALID, "k_bounds must increase strictly (index %d)", i);
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  GridHost g;
  g.N = n_wp;
  g.ng = n_gauss;
  g.kb.assign(k_bounds_host, k_bounds_host + n_wp + 1);
  std::vector<double> x, w;
  gauss_legendre(n_gauss, x, w);
  const int N = n_wp, ng = n_gauss;
  // Free packets (Sec. 3.1): momentum packets f(k) = 1, N_i = dk_i; energy
  // packets f(k) = sqrt(k/mu), N_i = dE_i, which in these units (E = k^2,
  // 2 mu = 1) is f(k) = sqrt(2k), N_i = k_i^2 - k_{i-1}^2.  Per bin the grid
  // keeps H0's diagonal <x_i|k^2|x_i> (momentum: (a^2 + ab + b^2)/3; energy:
  // the energy midpoint (a^2 + b^2)/2, the eigenvalue the paper gives), the
  // on-shell momentum q_i whose energy is the packet's free eigenvalue
  // (momentum: the midpoint; energy: sqrt of the energy midpoint), the
  // projection weights w k f(k) and 1/sqrt(N_i), and N_i/f(q_i)^2, the factor
  // of t(q,q) = f(q)^2 T_ii/(N_i q^2).
  const bool energy = packet == WPCD_PACKET_ENERGY;
  std::vector<double> eb(N + 1), dk(N), kbar(N), e0(N), wk((size_t)N * ng), rsdk(N);
  g.nodes.resize((size_t)N * ng);
  g.weights.resize((size_t)N * ng);
  for (int j = 0; j <= N; ++j) eb[j] = g.kb[j] * g.kb[j];
  for (int i = 0; i < N; ++i) {
    const double a = g.kb[i], b = g.kb[i + 1];
    if (energy) {
      const double dE = b * b - a * a;
      e0[i] = 0.5 * (a * a + b * b);
      kbar[i] = sqrt(e0[i]);
      dk[i] = dE / (2.0 * kbar[i]);
      rsdk[i] = 1.0 / sqrt(dE);
    } else {
      dk[i] = b - a;
      kbar[i] = 0.5 * (a + b);
      e0[i] = (a * a + a * b + b * b) / 3.0;  // bin average of k^2
      rsdk[i] = 1.0 / sqrt(dk[i]);
    }
    for (int q = 0; q < ng; ++q) {
      const double node = 0.5 * (b - a) * x[q] + 0.5 * (b + a);
      const double wt = 0.5 * (b - a) * w[q];
      g.nodes[(size_t)i * ng + q] = node;
      g.weights[(size_t)i * ng + q] = wt;
      wk[(size_t)i * ng + q] = energy ? wt * node * sqrt(2.0 * node) : wt * node;
    }
  }
  const size_t total = (size_t)(N + 1) * 2 + (size_t)N * 4 + (size_t)N * ng;
  std::vector<double> host(total);
  size_t o = 0;
  auto put = [&](const std::vector<double>& v) {
    const size_t at = o;
    std::copy(v.begin(), v.end(), host.begin() + o);
    o += v.size();
    return at;
  };
  const size_t o_kb = put(g.kb), o_eb = put(eb), o_dk = put(dk), o_kbar = put(kbar), o_e0 = put(e0), o_wk = put(wk),
               o_rs = put(rsdk);
  WPCD_HIP(hipMalloc(&g.dbuf, total * sizeof(double)), "hipMalloc(grid)");
  hipError_t e = hipMemcpy(g.dbuf, host.data(), total * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(g.dbuf);
    return hip_fail(e, "hipMemcpy(grid)");
  }
  g.dev = GridDev{g.dbuf + o_kb, g.dbuf + o_eb, g.dbuf + o_dk, g.dbuf + o_kbar, g.dbuf + o_e0, g.dbuf + o_wk,
                  g.dbuf + o_rs, N, ng};
  ctx->grids.push_back(std::move(g));
  *grid_id = (int)ctx->grids.size() - 1;
  return WPCD_OK;
}

int wpcd_grid_nodes(wpcd_ctx ctx, int grid_id, double* nodes_host, double* weights_host) {
  if (!ctx || grid_id < 0 || grid_id >= (int)ctx->grids.size())
    return fail(WPCD_ERR_INVALID, "wpcd_grid_nodes: bad context or grid id");
  const GridHost& g = ctx->grids[grid_id];
  if (nodes_host) std::copy(g.nodes.begin(), g.nodes.end(), nodes_host);
  if (weights_host) std::copy(g.weights.begin(), g.weights.end(), weights_host);
  return WPCD_OK;
}

void wpcd_batch_destroy(wpcd_batch b) {
  if (!b) return;
  hipSetDevice(b->device);
  hipFree(b->d_items);
  hipFree(b->d_grids);
  hipFree(b->d_sample_ptr);
  hipFree(b->d_sample_items);
  hipFree(b->d_x32);
  hipFree(b->d_work);
  hipFree(b->d_cl);
  hipFree(b->d_lam);
  hipFree(b->d_class);
  hipFree(b->d_jlist);
  hipFree(b->d_ref);
  hipFree(b->d_cand);
  hipFree(b->d_pick);
  hipFree(b->d_sig);
  hipFree(b->d_bases);
  jac_feedback_destroy(b->jfb);
  delete b;
}

int wpcd_batch_create(wpcd_ctx ctx, const wpcd_item* items_host, int n_items, wpcd_batch* out) {
  if (!ctx || !items_host || !out) return fail(WPCD_ERR_INVALID, "wpcd_batch_create: NULL argument");
  *out = nullptr;
  if (n_items < 1) return fail(WPCD_ERR_INVALID, "wpcd_batch_create: n_items must be >= 1");
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  wpcd_batch_s* b = new (std::nothrow) wpcd_batch_s;
  if (!b) return fail(WPCD_ERR_NOMEM, "wpcd_batch_create: host allocation");
  b->ctx = ctx;
  b->device = ctx->device;
  b->n_items = n_items;
  b->h_items.resize(n_items);
  int max_sample = -1;
  for (int i = 0; i < n_items; ++i) {
    const wpcd_item& in = items_host[i];
    if (in.grid_id < 0 || in.grid_id >= (int)ctx->grids.size()) {
      delete b;
      return fail(WPCD_ERR_INVALID, "item %d: unknown grid id %d", i, in.grid_id);
    }
    if (in.n_ch != 1 && in.n_ch != 2) {
      delete b;
      return fail(WPCD_ERR_INVALID, "item %d: n_ch must be 1 or 2", i);
    }
    if (in.J < 0 || (in.n_ch == 2 && in.J < 1) || in.sample_id < 0) {
      delete b;
      return fail(WPCD_ERR_INVALID, "item %d: need J >= 0 (>= 1 if coupled) and sample_id >= 0", i);
    }
    if (in.basis_id < -1 || in.basis_id >= (int)ctx->bases.size()) {
      delete b;
      return fail(WPCD_ERR_INVALID, "item %d: unknown basis id %d", i, in.basis_id);
    }
    if (in.basis_id >= 0 &&
        (ctx->bases[in.basis_id].grid != in.grid_id || ctx->bases[in.basis_id].nch != in.n_ch)) {
      delete b;
      return fail(WPCD_ERR_INVALID, "item %d: basis %d was registered for another grid or n_ch", i, in.basis_id);
    }
    const GridHost& g = ctx->grids[in.grid_id];
    const int n = in.n_ch * g.N;
    if (n > kMaxN) {
      delete b;
      return fail(WPCD_ERR_UNSUPPORTED, "item %d: n = %d exceeds %d", i, n, kMaxN);
    }
    ItemDev& d = b->h_items[i];
    d.grid = in.grid_id;
    d.nch = in.n_ch;
    d.N = g.N;
    d.n = n;
    d.ng = g.ng;
    d.J = in.J;
    d.sample = in.sample_id;
    d.basis = in.basis_id;
    // spin and orbital momenta (needed by wpcd_saclay only): S = -1 leaves them unset
    if (in.S != -1) {
      const bool ok = in.n_ch == 2 ? (in.S == 1 && in.l == in.J - 1)
                                   : ((in.S == 0 && in.l == in.J) || (in.S == 1 && in.l >= 0 && (in.l == in.J ||
                                       (in.J == 0 && in.l == 1))));
      if (!ok) {
        delete b;
        return fail(WPCD_ERR_INVALID, "item %d: (S, l, J) = (%d, %d, %d) is not a channel of a spin-1/2 pair "
                                      "(uncoupled: l = J, or 3P0; coupled: S = 1, l = J - 1)", i, in.S, in.l, in.J);
      }
      d.spin = in.S;
      d.l0 = in.l;
    } else {
      d.spin = -1;
      d.l0 = -1;
    }
    const int64_t M = in.basis_id >= 0 ? 0 : (int64_t)n * g.ng;
    d.u_off = b->u_elems;
    d.c_off = b->coef_elems;
    if (in.basis_id >= 0) {
      b->coef_elems += ctx->bases[in.basis_id].n_terms;
      b->n_affine++;
    } else {
      b->n_fine++;
    }
    d.v_off = b->v_elems;
    d.e_off = b->eval_elems;
    d.t_off = b->t_doubles;
    d.d_off = b->delta_elems;
    d.m_off = b->mix_elems;
    d.w_off = b->work_doubles;
    b->u_elems += M * M;
    b->v_elems += (int64_t)n * n;
    b->eval_elems += n;
    b->t_doubles += 2LL * g.N * in.n_ch * in.n_ch;
    b->delta_elems += (int64_t)g.N * in.n_ch;
    b->mix_elems += g.N;
    b->work_doubles += eig_work_doubles(n);
    b->max_n = std::max(b->max_n, n);
    b->min_n = b->min_n == 0 ? n : std::min(b->min_n, n);
    b->max_nbins = std::max(b->max_nbins, g.N);
    max_sample = std::max(max_sample, in.sample_id);
  }
  b->n_samples = max_sample + 1;
  // per-sample item lists (CSR)
  std::vector<int32_t> sptr(b->n_samples + 1, 0), sitems(n_items);
  for (int i = 0; i < n_items; ++i) sptr[items_host[i].sample_id + 1]++;
  for (int s = 0; s < b->n_samples; ++s) sptr[s + 1] += sptr[s];
  {
    std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
    for (int i = 0; i < n_items; ++i) sitems[fill[items_host[i].sample_id]++] = i;
  }
  // size classes of the eigensolver
  std::vector<int32_t> cls(n_items);
  {
    int cnt[kNumClasses] = {0};
    for (int i = 0; i < n_items; ++i) {
      const int c = size_class(b->h_items[i].n);
      cnt[c]++;
      b->class_maxn[c] = std::max(b->class_maxn[c], b->h_items[i].n);
    }
    for (int c = 0; c < kNumClasses; ++c) b->class_ptr[c + 1] = b->class_ptr[c] + cnt[c];
    int fill[kNumClasses];
    for (int c = 0; c < kNumClasses; ++c) fill[c] = b->class_ptr[c];
    for (int i = 0; i < n_items; ++i) cls[fill[size_class(b->h_items[i].n)]++] = i;
  }
  // warm-start lists: per size class, each group's first item starts cold,
  // and in the LDS classes further items up to one per compute unit do too
  // (they would otherwise wait for the references); the rest of a group
  // starts from its first item's eigenvectors
  constexpr int L = wpcd_batch_s::kC;
  std::vector<int32_t> ref(n_items, -1);
  std::vector<int32_t> seg[2 * L + 1];
  std::vector<int32_t> cand, pick;  // reference candidates and pick tasks (jlist offsets relative to the class)
  std::vector<int> pick_cls;
  {
    int n_cu = 256;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n_cu < 1)
      n_cu = 256;
    const bool warm = ctx->cfg.jacobi_start == 0;
    for (int c = 0; c < L; ++c) {
      const int cold_cap = c < L - 1 ? n_cu : 0;
      std::map<std::tuple<int, int, int, int>, int> first;  // group key -> its first (reference) item
      std::vector<int32_t> rest;
      for (int q = b->class_ptr[c]; q < b->class_ptr[c + 1]; ++q) {
        const int i = cls[q];
        const ItemDev& d = b->h_items[i];
        const auto key = std::make_tuple(d.grid, d.nch, d.J, d.basis);
        if (!warm || first.emplace(key, i).second)
          seg[c].push_back(i);
        else
          rest.push_back(i);
      }
      for (int32_t i : rest) {
        if ((int)seg[c].size() < cold_cap) {
          seg[c].push_back(i);
        } else {
          const ItemDev& d = b->h_items[i];
          ref[i] = first[std::make_tuple(d.grid, d.nch, d.J, d.basis)];
          seg[L + c].push_back(i);
        }
      }
      if (c < L - 1 && !seg[L + c].empty()) {
        // LDS classes: the warm items of a group take the group's cold item
        // nearest in V (chosen on the device; ref[] keeps the group's first
        // item until then); warm items ordered by group, in runs of <= 16
        std::map<std::tuple<int, int, int, int>, std::vector<int32_t>> cold_of, warm_of;
        for (int32_t i : seg[c]) {
          const ItemDev& d = b->h_items[i];
          cold_of[std::make_tuple(d.grid, d.nch, d.J, d.basis)].push_back(i);
        }
        for (int32_t i : seg[L + c]) {
          const ItemDev& d = b->h_items[i];
          warm_of[std::make_tuple(d.grid, d.nch, d.J, d.basis)].push_back(i);
        }
        seg[L + c].clear();
        for (auto& kv : warm_of) {
          const std::vector<int32_t>& cl_items = cold_of[kv.first];
          const int coff = (int)cand.size();
          cand.insert(cand.end(), cl_items.begin(), cl_items.end());
          for (size_t w0 = 0; w0 < kv.second.size(); w0 += kWarmPick) {
            const int cnt = (int)std::min<size_t>(kWarmPick, kv.second.size() - w0);
            pick.insert(pick.end(), {(int32_t)(seg[L + c].size() + w0), cnt, coff, (int32_t)cl_items.size()});
            pick_cls.push_back(c);
          }
          seg[L + c].insert(seg[L + c].end(), kv.second.begin(), kv.second.end());
        }
      }
    }
    for (int c = 0; c < L; ++c)
      for (int32_t i : seg[L + c]) {
        const int n = b->h_items[i].n;
        b->warm_min_n = b->warm_min_n == 0 ? n : std::min(b->warm_min_n, n);
        b->warm_max_n = std::max(b->warm_max_n, n);
      }
    std::vector<char> is_ref(n_items, 0);
    for (int i = 0; i < n_items; ++i)
      if (ref[i] >= 0 && !is_ref[ref[i]]) {
        is_ref[ref[i]] = 1;
        seg[2 * L].push_back(ref[i]);
      }
    for (int32_t i : cand)
      if (!is_ref[i]) {
        is_ref[i] = 1;
        seg[2 * L].push_back(i);
      }
  }
  std::vector<int32_t> jlist;
  for (int t = 0; t <= 2 * L; ++t) {
    b->jl_ptr[t] = (int)jlist.size();
    jlist.insert(jlist.end(), seg[t].begin(), seg[t].end());
  }
  b->jl_ptr[2 * L + 1] = (int)jlist.size();
  for (size_t t = 0; t < pick_cls.size(); ++t) pick[4 * t] += b->jl_ptr[L + pick_cls[t]];
  b->n_pick = (int)pick_cls.size();
  std::vector<GridDev> gd(ctx->grids.size());
  for (size_t i = 0; i < gd.size(); ++i) gd[i] = ctx->grids[i].dev;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes > 0 ? bytes : 1);
  };
  alloc((void**)&b->d_items, sizeof(ItemDev) * n_items);
  alloc((void**)&b->d_grids, sizeof(GridDev) * gd.size());
  alloc((void**)&b->d_sample_ptr, sizeof(int32_t) * sptr.size());
  alloc((void**)&b->d_sample_items, sizeof(int32_t) * sitems.size());
  alloc((void**)&b->d_x32, sizeof(float) * b->v_elems);
  alloc((void**)&b->d_work, sizeof(double) * b->work_doubles);
  alloc((void**)&b->d_cl, sizeof(int32_t) * b->eval_elems);
  alloc((void**)&b->d_lam, sizeof(double) * b->eval_elems);
  alloc((void**)&b->d_class, sizeof(int32_t) * n_items);
  alloc((void**)&b->d_jlist, sizeof(int32_t) * jlist.size());
  alloc((void**)&b->d_ref, sizeof(int32_t) * n_items);
  alloc((void**)&b->d_cand, sizeof(int32_t) * cand.size());
  alloc((void**)&b->d_pick, sizeof(int32_t) * pick.size());
  alloc((void**)&b->d_sig, b->n_pick > 0 ? sizeof(float) * kWarmSig * (size_t)n_items : 0);
  std::vector<BasisDev> bd(ctx->bases.size());
  for (size_t i = 0; i < bd.size(); ++i) bd[i] = BasisDev{ctx->bases[i].dbuf, ctx->bases[i].n, ctx->bases[i].n_terms};
  alloc((void**)&b->d_bases, sizeof(BasisDev) * bd.size());
  if (e == hipSuccess && !bd.empty())
    e = hipMemcpy(b->d_bases, bd.data(), sizeof(BasisDev) * bd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_items, b->h_items.data(), sizeof(ItemDev) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_grids, gd.data(), sizeof(GridDev) * gd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_sample_ptr, sptr.data(), sizeof(int32_t) * sptr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_sample_items, sitems.data(), sizeof(int32_t) * sitems.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_class, cls.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess && !jlist.empty())
    e = hipMemcpy(b->d_jlist, jlist.data(), sizeof(int32_t) * jlist.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_ref, ref.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess && !cand.empty())
    e = hipMemcpy(b->d_cand, cand.data(), sizeof(int32_t) * cand.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pick.empty())
    e = hipMemcpy(b->d_pick, pick.data(), sizeof(int32_t) * pick.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = jac_feedback_create(b->jfb);
  if (e != hipSuccess) {
    wpcd_batch_destroy(b);
    return hip_fail(e, "wpcd_batch_create");
  }
  *out = b;
  return WPCD_OK;
}

int wpcd_batch_layout_get(wpcd_batch b, wpcd_batch_layout* out) {
  if (!b || !out) return fail(WPCD_ERR_INVALID, "wpcd_batch_layout_get: NULL argument");
  out->u_elems = b->u_elems;
  out->v_elems = b->v_elems;
  out->eval_elems = b->eval_elems;
  out->t_doubles = b->t_doubles;
  out->delta_elems = b->delta_elems;
  out->mix_elems = b->mix_elems;
  out->coef_elems = b->coef_elems;
  out->n_items = b->n_items;
  out->n_samples = b->n_samples;
  out->max_n = b->max_n;
  out->max_nbins = b->max_nbins;
  return WPCD_OK;
}

int wpcd_batch_offsets(wpcd_batch b, int64_t* u_off, int64_t* v_off, int64_t* eval_off, int64_t* t_off,
                       int64_t* delta_off, int64_t* mix_off, int64_t* coef_off) {
  if (!b) return fail(WPCD_ERR_INVALID, "wpcd_batch_offsets: NULL batch");
  for (int i = 0; i < b->n_items; ++i) {
    const ItemDev& d = b->h_items[i];
    if (u_off) u_off[i] = d.u_off;
    if (v_off) v_off[i] = d.v_off;
    if (eval_off) eval_off[i] = d.e_off;
    if (t_off) t_off[i] = d.t_off;
    if (delta_off) delta_off[i] = d.d_off;
    if (mix_off) mix_off[i] = d.m_off;
    if (coef_off) coef_off[i] = d.c_off;
  }
  return WPCD_OK;
}

int wpcd_project(wpcd_batch b, const void* u_fine, int u_dtype, double* v64, hipStream_t stream) {
  if (!b || !u_fine || !v64) return fail(WPCD_ERR_INVALID, "wpcd_project: NULL argument");
  if (u_dtype != WPCD_DTYPE_F32 && u_dtype != WPCD_DTYPE_F64)
    return fail(WPCD_ERR_INVALID, "wpcd_project: unknown u_dtype %d", u_dtype);
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  if (b->n_fine == 0) return WPCD_OK;
  const int elem = u_dtype == WPCD_DTYPE_F32 ? 4 : 8;
  bool generic = false;
  for (const ItemDev& it : b->h_items) generic = generic || (it.basis < 0 && !project_tiled(it, u_fine, elem));
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_PROJECT, stream,
                 [&] { return launch_project(b->d_items, b->n_items, b->max_n, b->d_grids, u_fine, u_dtype, v64,
                                       generic, stream); }),
           "wpcd_project launch");
  return WPCD_OK;
}

int wpcd_project_affine(wpcd_batch b, const double* coef, double* v64, hipStream_t stream) {
  if (!b || !v64 || (!coef && b->coef_elems > 0)) return fail(WPCD_ERR_INVALID, "wpcd_project_affine: NULL argument");
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  if (b->n_affine == 0) return WPCD_OK;
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_PROJECT, stream,
                 [&] {
                   return launch_project_affine(b->d_items, b->n_items, b->max_n, b->d_bases, coef, v64, stream);
                 }),
           "wpcd_project_affine launch");
  return WPCD_OK;
}

int wpcd_basis_register(wpcd_ctx ctx, int grid_id, int n_ch, int n_terms, const void* u_terms, int u_dtype,
                        hipStream_t stream, int* basis_id) {
  if (!ctx || !u_terms || !basis_id) return fail(WPCD_ERR_INVALID, "wpcd_basis_register: NULL argument");
  if (grid_id < 0 || grid_id >= (int)ctx->grids.size())
    return fail(WPCD_ERR_INVALID, "wpcd_basis_register: unknown grid id %d", grid_id);
  if (n_ch != 1 && n_ch != 2) return fail(WPCD_ERR_INVALID, "wpcd_basis_register: n_ch must be 1 or 2");
  if (n_terms < 1 || n_terms > 16) return fail(WPCD_ERR_INVALID, "wpcd_basis_register: n_terms must be in [1, 16]");
  if (u_dtype != WPCD_DTYPE_F32 && u_dtype != WPCD_DTYPE_F64)
    return fail(WPCD_ERR_INVALID, "wpcd_basis_register: unknown u_dtype %d", u_dtype);
  const GridHost& g = ctx->grids[grid_id];
  const int n = n_ch * g.N;
  if (n > kMaxN) return fail(WPCD_ERR_UNSUPPORTED, "wpcd_basis_register: n = %d exceeds %d", n, kMaxN);
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const int64_t M = (int64_t)n * g.ng;
  // the terms as items of a temporary batch over a one-entry grid table
  std::vector<ItemDev> it(n_terms);
  for (int t = 0; t < n_terms; ++t) {
    ItemDev& d = it[t];
    memset(&d, 0, sizeof(d));
    d.grid = 0;
    d.nch = n_ch;
    d.N = g.N;
    d.n = n;
    d.ng = g.ng;
    d.basis = -1;
    d.u_off = t * M * M;
    d.v_off = (int64_t)t * n * n;
  }
  BasisHost bh;
  bh.grid = grid_id;
  bh.nch = n_ch;
  bh.n = n;
  bh.n_terms = n_terms;
  ItemDev* d_it = nullptr;
  GridDev* d_g = nullptr;
  const char* what = "wpcd_basis_register: allocation";
  hipError_t e = hipMalloc((void**)&bh.dbuf, sizeof(double) * n_terms * (size_t)n * n);
  if (e == hipSuccess) e = hipMalloc((void**)&d_it, sizeof(ItemDev) * n_terms);
  if (e == hipSuccess) e = hipMalloc((void**)&d_g, sizeof(GridDev));
  if (e == hipSuccess) {
    what = "wpcd_basis_register: upload";
    e = hipMemcpy(d_it, it.data(), sizeof(ItemDev) * n_terms, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(d_g, &g.dev, sizeof(GridDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    what = "wpcd_basis_register: projection launch";
    e = launch_project(d_it, n_terms, n, d_g, u_terms, u_dtype, bh.dbuf, true, stream);
  }
  if (e == hipSuccess) {
    what = "wpcd_basis_register: projection";
    e = hipStreamSynchronize(stream);
  }
  hipFree(d_it);
  hipFree(d_g);
  if (e != hipSuccess) {
    hipFree(bh.dbuf);
    return hip_fail(e, what);
  }
  ctx->bases.push_back(bh);
  *basis_id = (int)ctx->bases.size() - 1;
  return WPCD_OK;
}

// The second stream of the batch path and its fork/join events, created on
// first use (the request loop never needs them, and every stream takes a
// share of the hardware queues its own streams use).  All three or none: a
// partial set would pass null events to later calls.
static int ensure_side(wpcd_ctx ctx) {
  if (ctx->side != nullptr) return WPCD_OK;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (join) hipEventDestroy(join);
    if (fork) hipEventDestroy(fork);
    if (side) hipStreamDestroy(side);
    return dev_fail(ctx, e, "wpcd_eigh: second stream and its events");
  }
  ctx->side = side;
  ctx->fork = fork;
  ctx->join = join;
  return WPCD_OK;
}

// Eigensolver work-space of one call: FP32 eigenvectors (v_elems floats), the
// per-item FP64 work-space (work_doubles), cluster lists and Rayleigh
// quotients (eval_elems each) and the warm-start samples (kWarmSig floats per
// item, when the batch has pick tasks).
struct EighBufs {
  float* x32;
  double* work;
  int32_t* cl;
  double* lam;
  float* sig;
};

// wpcd_eigh after its argument checks.  concurrent: the batch path proper
// (second stream for the reference choice and part of the refinement, stage
// timers); otherwise every launch goes to `stream` and nothing is timed, so
// the call creates no stream, event or allocation.
static int eigh_run(wpcd_batch b, const double* v64, int mode, double* eval, double* evec, int32_t* status,
                    hipStream_t stream, const EighBufs& w, bool concurrent) {
  const wpcd_config& c = b->ctx->cfg;
  auto stage = [&](int st, auto launch) -> hipError_t {
    return concurrent ? timed(b->ctx, st, stream, launch) : launch();
  };
  if (mode == WPCD_MIXED) {
    if (concurrent) {
      const int rc = ensure_side(b->ctx);
      if (rc != WPCD_OK) return rc;
    }
    hipStream_t side = concurrent ? b->ctx->side : nullptr;
    // one FP32 Jacobi launch per size class: LDS-resident up to n = kMaxLdsN,
    // device memory above
    {
      constexpr int L = wpcd_batch_s::kC;
      unsigned long long* cnt = (concurrent && b->ctx->profiling) ? b->ctx->d_counters : nullptr;
      // one timed group per launch of the LDS kernel (per launch sequence of
      // the device-memory Jacobi)
      auto solve = [&](int seg, int k, const int32_t* ref) -> hipError_t {
        const int n_sel = b->jl_ptr[seg + 1] - b->jl_ptr[seg];
        if (n_sel == 0) return hipSuccess;
        const int32_t* sel = b->d_jlist + b->jl_ptr[seg];
        return stage(WPCD_STAGE_JACOBI_F32, [&] {
          if (k < L - 1)
            return launch_jacobi_f32_lds(b->d_items, sel, n_sel, b->class_maxn[k], b->d_grids, v64, w.x32, eval,
                                         status, c.max_sweeps, (float)c.jacobi_tol_f32, (float)c.jacobi_stop_f32,
                                         c.jacobi_block, ref, w.work, cnt, stream);
          return launch_jacobi_global(1, b->d_items, sel, n_sel, b->class_maxn[k], b->d_grids, v64, w.work, evec,
                                      w.x32, eval, status, c.max_sweeps, c.jacobi_tol_f32, c.jacobi_stop_f32, ref,
                                      &b->jfb, stream);
        });
      };
      // cold starts (each group's reference among them), then the warm starts
      // from the references' eigenvectors; the choice of references (V only)
      // runs on the side stream beside the cold Jacobi
      const int n_warm = b->jl_ptr[2 * L] - b->jl_ptr[L];
      const bool side_pick = side != nullptr && n_warm > 0 && b->n_pick > 0;
      if (side_pick) {
        WPCD_HIPX(b->ctx, hipEventRecord(b->ctx->fork, stream), "wpcd_eigh: fork");
        WPCD_HIPX(b->ctx, hipStreamWaitEvent(side, b->ctx->fork, 0), "wpcd_eigh: fork");
        WPCD_HIPX(b->ctx, launch_warm_pick(b->d_items, b->n_items, b->d_jlist, b->d_pick, b->n_pick, b->d_cand, w.sig,
                                           v64, b->d_ref, side),
                  "wpcd_eigh: reference choice launch");
        WPCD_HIPX(b->ctx, hipEventRecord(b->ctx->join, side), "wpcd_eigh: join");
      }
      for (int k = 0; k < L; ++k) WPCD_HIPX(b->ctx, solve(k, k, nullptr), "wpcd_eigh: FP32 Jacobi launch");
      if (side_pick) WPCD_HIPX(b->ctx, hipStreamWaitEvent(stream, b->ctx->join, 0), "wpcd_eigh: join");
      if (n_warm > 0) {
        WPCD_HIPX(b->ctx, stage(WPCD_STAGE_WARM_PREP,
                                [&] {
                                  return launch_jacobi_warm_prep(
                                      b->d_items, b->n_items, b->d_jlist + b->jl_ptr[2 * L],
                                      b->jl_ptr[2 * L + 1] - b->jl_ptr[2 * L], b->d_jlist + b->jl_ptr[L], n_warm,
                                      b->d_ref, b->warm_min_n, b->warm_max_n, b->d_jlist, b->d_pick,
                                      side_pick ? 0 : b->n_pick, b->d_cand, w.sig, b->d_grids, v64, w.x32, w.work,
                                      stream);
                                }),
                  "wpcd_eigh: warm-start preparation launch");
      }
      for (int k = 0; k < L; ++k) WPCD_HIPX(b->ctx, solve(L + k, k, b->d_ref), "wpcd_eigh: FP32 Jacobi launch");
    }
    WPCD_HIPX(b->ctx, stage(WPCD_STAGE_REFINE,
                            [&] {
                              return launch_refine(b->d_items, b->n_items, b->min_n, b->max_n, b->d_grids, v64, w.x32,
                                                   evec, eval, w.lam, w.work, w.cl, status, c.refine_steps,
                                                   c.refine_close_log10, c.refine_gemm, c.refine_rr_steps, stream, side,
                                                   b->ctx->fork, b->ctx->join);
                            }),
              "wpcd_eigh: FP64 refinement launch");
  } else {
    WPCD_HIPX(b->ctx, stage(WPCD_STAGE_JACOBI_F64,
                            [&] {
                              return launch_jacobi_global(0, b->d_items, nullptr, b->n_items, b->max_n, b->d_grids,
                                                          v64, w.work, evec, w.x32, eval, status, c.max_sweeps,
                                                          c.jacobi_tol_f64, 8.0 * c.jacobi_tol_f64, nullptr,
                                                          &b->jfb, stream);
                            }),
              "wpcd_eigh: FP64 Jacobi launch");
  }
  return WPCD_OK;
}

// Argument checks shared by wpcd_eigh and wpcd_eigh_noalloc.
static int eigh_check(wpcd_batch b, const double* v64, int mode, const double* eval, const double* evec,
                      const int32_t* status, const char* who) {
  if (!b || !v64 || !eval || !evec || !status) return fail(WPCD_ERR_INVALID, "%s: NULL argument", who);
  if (mode != WPCD_MIXED && mode != WPCD_F64) return fail(WPCD_ERR_INVALID, "%s: unknown mode %d", who, mode);
  if (mode == WPCD_MIXED && b->ctx->cfg.refine_steps < 1)
    return fail(WPCD_ERR_UNSUPPORTED, "%s: WPCD_MIXED needs refine_steps >= 1", who);
  return WPCD_OK;
}

int wpcd_eigh(wpcd_batch b, const double* v64, int mode, double* eval, double* evec, int32_t* status,
              hipStream_t stream) {
  const int rc = eigh_check(b, v64, mode, eval, evec, status, "wpcd_eigh");
  if (rc != WPCD_OK) return rc;
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  return eigh_run(b, v64, mode, eval, evec, status, stream, EighBufs{b->d_x32, b->d_work, b->d_cl, b->d_lam, b->d_sig},
                  true);
}

int wpcd_eigh_noalloc(wpcd_batch b, const double* v64, int mode, double* eval, double* evec, int32_t* status,
                      hipStream_t stream) {
  const int rc = eigh_check(b, v64, mode, eval, evec, status, "wpcd_eigh_noalloc");
  if (rc != WPCD_OK) return rc;
  const ScratchPlan sp = scratch_plan(b);
  if (sp.total > kScratchBytes)
    return fail(WPCD_ERR_UNSUPPORTED,
                "wpcd_eigh_noalloc: the batch needs %zu bytes of eigensolver scratch, the static scratch holds %zu "
                "(split the batch or use wpcd_eigh)",
                sp.total, kScratchBytes);
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  unsigned char* base = scratch_ptr(b->ctx->device);
  if (!base) return fail(WPCD_ERR_DEVICE, "wpcd_eigh_noalloc: %s", scratch_error(b->ctx->device));
  const EighBufs w{reinterpret_cast<float*>(base + sp.x32), reinterpret_cast<double*>(base + sp.work),
                   reinterpret_cast<int32_t*>(base + sp.cl), reinterpret_cast<double*>(base + sp.lam),
                   reinterpret_cast<float*>(base + sp.sig)};
  return eigh_run(b, v64, mode, eval, evec, status, stream, w, false);
}

int wpcd_tmatrix(wpcd_batch b, const double* v64, const double* eval, const double* evec, int mode, double* t,
                 int32_t* status, hipStream_t stream) {
  if (!b || !v64 || !eval || !evec || !t || !status) return fail(WPCD_ERR_INVALID, "wpcd_tmatrix: NULL argument");
  if (mode != WPCD_MIXED && mode != WPCD_F64) return fail(WPCD_ERR_INVALID, "wpcd_tmatrix: unknown mode %d", mode);
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_TMATRIX, stream,
                 [&] {
                   return launch_tmatrix(b->d_items, b->n_items, b->max_n, b->d_grids, v64, eval, evec, mode, t, status,
                                         stream);
                 }),
           "wpcd_tmatrix launch");
  return WPCD_OK;
}

int wpcd_observables(wpcd_batch b, const double* t, double* delta_deg, double* mix_deg, double* s_dev,
                     hipStream_t stream) {
  if (!b || !t || !delta_deg || !mix_deg) return fail(WPCD_ERR_INVALID, "wpcd_observables: NULL argument");
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_OBSERVABLES, stream,
                 [&] {
                   return launch_observables(b->d_items, b->n_items, b->max_nbins, b->d_grids, t, delta_deg, mix_deg,
                                             s_dev, stream);
                 }),
           "wpcd_observables launch");
  return WPCD_OK;
}

int wpcd_saclay(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev, int n_tlab,
                const double* theta_deg, int n_theta, double* amp, double* dsdo_mb, hipStream_t stream) {
  if (!b || !delta_deg || !mix_deg || !tlab_mev || !theta_deg || !dsdo_mb)
    return fail(WPCD_ERR_INVALID, "wpcd_saclay: NULL argument");
  if (n_tlab < 1 || n_theta < 1 || (int64_t)n_tlab * n_theta > 1024)
    return fail(WPCD_ERR_INVALID, "wpcd_saclay: need n_tlab, n_theta >= 1 and n_tlab * n_theta <= 1024");
  if (b->max_nbins > 1200) return fail(WPCD_ERR_UNSUPPORTED, "wpcd_saclay: more than 1200 bins");
  for (int i = 0; i < b->n_items; ++i)
    if (b->h_items[i].spin < 0)
      return fail(WPCD_ERR_INVALID, "wpcd_saclay: item %d has no spin and orbital momentum (wpcd_item.S, .l)", i);
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  WPCD_HIPX(b->ctx,
            timed(b->ctx, WPCD_STAGE_SIGMA, stream,
                  [&] {
                    return launch_saclay(b->d_items, b->d_sample_ptr, b->d_sample_items, b->n_samples, b->d_grids,
                                         delta_deg, mix_deg, tlab_mev, n_tlab, theta_deg, n_theta, amp, dsdo_mb,
                                         stream);
                  }),
            "wpcd_saclay launch");
  return WPCD_OK;
}

int wpcd_sigma_tot(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev, int n_tlab,
                   double* sigma_mb, hipStream_t stream) {
  if (!b || !delta_deg || !mix_deg || !tlab_mev || !sigma_mb)
    return fail(WPCD_ERR_INVALID, "wpcd_sigma_tot: NULL argument");
  if (n_tlab < 1 || n_tlab > 1024) return fail(WPCD_ERR_INVALID, "wpcd_sigma_tot: n_tlab must be in [1, 1024]");
  if (b->max_nbins > 1200) return fail(WPCD_ERR_UNSUPPORTED, "wpcd_sigma_tot: more than 1200 bins");
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_SIGMA, stream,
                 [&] {
                   return launch_sigma(b->d_items, b->d_sample_ptr, b->d_sample_items, b->n_samples, b->d_grids,
                                       delta_deg, mix_deg, tlab_mev, nullptr, n_tlab, sigma_mb, stream);
                 }),
           "wpcd_sigma_tot launch");
  return WPCD_OK;
}

int wpcd_sigma_band(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev, int n_tlab,
                    const double* fracs, int n_frac, double* sigma_lo_mb, double* sigma_hi_mb, hipStream_t stream) {
  if (!b || !delta_deg || !mix_deg || !tlab_mev || !fracs || !sigma_lo_mb || !sigma_hi_mb)
    return fail(WPCD_ERR_INVALID, "wpcd_sigma_band: NULL argument");
  if (n_tlab < 1 || n_tlab > 256) return fail(WPCD_ERR_INVALID, "wpcd_sigma_band: n_tlab must be in [1, 256]");
  if (n_frac < 1 || n_frac > 16) return fail(WPCD_ERR_INVALID, "wpcd_sigma_band: n_frac must be in [1, 16]");
  if (b->max_nbins > 1200) return fail(WPCD_ERR_UNSUPPORTED, "wpcd_sigma_band: more than 1200 bins");
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  WPCD_HIPX(b->ctx, timed(b->ctx, WPCD_STAGE_SIGMA, stream,
                          [&] {
                            return launch_sigma_band(b->d_items, b->d_sample_ptr, b->d_sample_items, b->n_samples,
                                                     b->d_grids, delta_deg, mix_deg, tlab_mev, n_tlab, fracs, n_frac,
                                                     sigma_lo_mb, sigma_hi_mb, stream);
                          }),
            "wpcd_sigma_band launch");
  return WPCD_OK;
}

// ------------------------------------------------------- matrix inversion
void wpcd_mi_destroy(wpcd_mi m) {
  if (!m) return;
  hipSetDevice(m->device);
  hipFree(m->d_items);
  hipFree(m->d_pts);
  hipFree(m->d_qw);
  hipFree(m->d_loss);
  hipFree(m->d_sample_ptr);
  hipFree(m->d_sample_items);
  delete m;
}

int wpcd_mi_create(wpcd_ctx ctx, const wpcd_mi_item* items_host, int n_items, int n_q, double cutoff,
                   const double* tlab_host, int n_e, wpcd_mi* out) {
  if (!ctx || !items_host || !tlab_host || !out) return fail(WPCD_ERR_INVALID, "wpcd_mi_create: NULL argument");
  *out = nullptr;
  if (n_items < 1 || n_items > 65535) return fail(WPCD_ERR_INVALID, "wpcd_mi_create: n_items must be in [1, 65535]");
  if (n_e < 1 || n_e > 4096) return fail(WPCD_ERR_INVALID, "wpcd_mi_create: n_e must be in [1, 4096]");
  if (n_q < 2) return fail(WPCD_ERR_INVALID, "wpcd_mi_create: n_q must be >= 2");
  if (!(cutoff > 0.0) || !isfinite(cutoff)) return fail(WPCD_ERR_INVALID, "wpcd_mi_create: cutoff must be > 0");
  wpcd_mi_s* m = new (std::nothrow) wpcd_mi_s;
  if (!m) return fail(WPCD_ERR_NOMEM, "wpcd_mi_create: host allocation");
  m->ctx = ctx;
  m->device = ctx->device;
  m->n_items = n_items;
  m->nq = n_q;
  m->ne = n_e;
  m->cutoff = cutoff;
  int max_sample = -1;
  m->h_items.resize(n_items);
  for (int i = 0; i < n_items; ++i) {
    const wpcd_mi_item& in = items_host[i];
    if ((in.n_ch != 1 && in.n_ch != 2) || in.J < 0 || (in.n_ch == 2 && in.J < 1) || in.sample_id < 0) {
      delete m;
      return fail(WPCD_ERR_INVALID, "wpcd_mi_create: item %d: need n_ch 1 or 2, J >= 0 (>= 1 if coupled), "
                                    "sample_id >= 0", i);
    }
    MiItemDev& d = m->h_items[i];
    const int K = in.n_ch;
    d.nch = K;
    d.J = in.J;
    d.sample = in.sample_id;
    d.pad = 0;
    d.u_off = m->u_elems;
    d.k_off = m->k_elems;
    d.d_off = m->d_elems;
    d.m_off = m->m_elems;
    const int64_t lu = (int64_t)K * (n_q + n_e);
    m->u_elems += lu * lu;
    m->k_elems += (int64_t)n_e * K * K;
    m->d_elems += (int64_t)n_e * K;
    m->m_elems += n_e;
    m->max_nch = std::max(m->max_nch, K);
    max_sample = std::max(max_sample, in.sample_id);
  }
  m->n_samples = max_sample + 1;
  if (n_q > kMaxMiNq || mi_lds_bytes(n_q, m->max_nch) > 160 * 1024 - 4096) {
    delete m;
    return fail(WPCD_ERR_UNSUPPORTED, "wpcd_mi_create: n_q = %d too large for %s items (the system must fit the LDS)",
                n_q, m->max_nch == 2 ? "coupled" : "uncoupled");
  }
  // Gauss-Legendre nodes on [0, cutoff], then the on-shell momenta
  std::vector<double> x, w;
  gauss_legendre(n_q, x, w);
  m->pts.resize(n_q + n_e);
  m->wts.resize(n_q);
  for (int j = 0; j < n_q; ++j) {
    m->pts[j] = 0.5 * cutoff * (x[j] + 1.0);
    m->wts[j] = 0.5 * cutoff * w[j];
  }
  for (int e = 0; e < n_e; ++e) {
    const double t = tlab_host[e];
    const double p = sqrt(938.918 * t / 2.0) / 197.327;
    if (!(t > 0.0) || !(p < cutoff)) {
      delete m;
      return fail(WPCD_ERR_INVALID, "wpcd_mi_create: T_lab[%d] = %g gives p outside (0, cutoff)", e, t);
    }
    for (int j = 0; j < n_q; ++j)
      if (m->pts[j] == p) {
        delete m;
        return fail(WPCD_ERR_INVALID, "wpcd_mi_create: T_lab[%d] puts p on a quadrature node", e);
      }
    m->pts[n_q + e] = p;
  }
  std::vector<int32_t> sptr(m->n_samples + 1, 0), sitems(n_items);
  for (int i = 0; i < n_items; ++i) sptr[items_host[i].sample_id + 1]++;
  for (int s = 0; s < m->n_samples; ++s) sptr[s + 1] += sptr[s];
  {
    std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
    for (int i = 0; i < n_items; ++i) sitems[fill[items_host[i].sample_id]++] = i;
  }
  hipError_t e = hipSetDevice(ctx->device);
  auto alloc = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes > 0 ? bytes : 1);
  };
  alloc((void**)&m->d_items, sizeof(MiItemDev) * n_items);
  alloc((void**)&m->d_pts, sizeof(double) * m->pts.size());
  alloc((void**)&m->d_qw, sizeof(double) * n_q);
  alloc((void**)&m->d_loss, sizeof(double) * (size_t)n_items * n_e);
  alloc((void**)&m->d_sample_ptr, sizeof(int32_t) * sptr.size());
  alloc((void**)&m->d_sample_items, sizeof(int32_t) * sitems.size());
  if (e == hipSuccess) e = hipMemcpy(m->d_items, m->h_items.data(), sizeof(MiItemDev) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_pts, m->pts.data(), sizeof(double) * m->pts.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_qw, m->wts.data(), sizeof(double) * n_q, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_sample_ptr, sptr.data(), sizeof(int32_t) * sptr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_sample_items, sitems.data(), sizeof(int32_t) * sitems.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    wpcd_mi_destroy(m);
    return hip_fail(e, "wpcd_mi_create");
  }
  *out = m;
  return WPCD_OK;
}

int wpcd_mi_points(wpcd_mi m, double* points_host, double* weights_host) {
  if (!m) return fail(WPCD_ERR_INVALID, "wpcd_mi_points: NULL solver");
  if (points_host) std::copy(m->pts.begin(), m->pts.end(), points_host);
  if (weights_host) std::copy(m->wts.begin(), m->wts.end(), weights_host);
  return WPCD_OK;
}

int wpcd_mi_layout_get(wpcd_mi m, wpcd_mi_layout* out, int64_t* u_off_host, int64_t* k_off_host,
                       int64_t* delta_off_host, int64_t* mix_off_host) {
  if (!m) return fail(WPCD_ERR_INVALID, "wpcd_mi_layout_get: NULL solver");
  if (out) {
    out->u_elems = m->u_elems;
    out->kmat_elems = m->k_elems;
    out->delta_elems = m->d_elems;
    out->mix_elems = m->m_elems;
    out->n_items = m->n_items;
    out->n_samples = m->n_samples;
    out->n_q = m->nq;
    out->n_e = m->ne;
  }
  for (int i = 0; i < m->n_items; ++i) {
    const MiItemDev& d = m->h_items[i];
    if (u_off_host) u_off_host[i] = d.u_off;
    if (k_off_host) k_off_host[i] = d.k_off;
    if (delta_off_host) delta_off_host[i] = d.d_off;
    if (mix_off_host) mix_off_host[i] = d.m_off;
  }
  return WPCD_OK;
}

int wpcd_mi_solve(wpcd_mi m, const double* u, double* kmat, double* delta_deg, double* mix_deg, double* sigma_mb,
                  int32_t* status, hipStream_t stream) {
  if (!m || !u || !kmat || !delta_deg || !mix_deg || !status)
    return fail(WPCD_ERR_INVALID, "wpcd_mi_solve: NULL argument");
  WPCD_HIPX(m->ctx, hipSetDevice(m->ctx->device), "hipSetDevice");
  WPCD_STICKY(m->ctx);
  WPCD_HIPX(m->ctx,
            launch_mi_solve(m->d_items, m->n_items, m->nq, m->ne, m->max_nch, m->d_qw, m->d_pts, m->cutoff, u, kmat,
                            delta_deg, mix_deg, m->d_loss, m->d_sample_ptr, m->d_sample_items,
                            sigma_mb ? m->n_samples : 0, sigma_mb, status, stream),
            "wpcd_mi_solve launch");
  return WPCD_OK;
}

// ------------------------------------------------------------ whole path
int wpcd_run(wpcd_batch b, const wpcd_path_args* a, int mode, hipStream_t stream) {
  if (!b || !a) return fail(WPCD_ERR_INVALID, "wpcd_run: NULL argument");
  if (b->n_fine > 0 && !a->u_fine) return fail(WPCD_ERR_INVALID, "wpcd_run: the batch has fine-mesh items but no u_fine");
  if (b->n_affine > 0 && !a->coef) return fail(WPCD_ERR_INVALID, "wpcd_run: the batch has basis items but no coef");
  if (a->n_tlab > 0 && (!a->tlab_mev || !a->sigma_mb)) return fail(WPCD_ERR_INVALID, "wpcd_run: n_tlab > 0 needs tlab and sigma");
  int rc = WPCD_OK;
  if (b->n_fine > 0) rc = wpcd_project(b, a->u_fine, a->u_dtype, a->v64, stream);
  if (rc == WPCD_OK && b->n_affine > 0) rc = wpcd_project_affine(b, a->coef, a->v64, stream);
  if (rc == WPCD_OK) rc = wpcd_eigh(b, a->v64, mode, a->eval, a->evec, a->eig_status, stream);
  if (rc == WPCD_OK) rc = wpcd_tmatrix(b, a->v64, a->eval, a->evec, mode, a->t, a->t_status, stream);
  if (rc == WPCD_OK) rc = wpcd_observables(b, a->t, a->delta_deg, a->mix_deg, a->s_dev, stream);
  if (rc == WPCD_OK && a->n_tlab > 0)
    rc = wpcd_sigma_tot(b, a->delta_deg, a->mix_deg, a->tlab_mev, a->n_tlab, a->sigma_mb, stream);
  return rc;
}

// ------------------------------------------------------------- autotuner
// Signature of a batch for the tune cache: mode and, per eigensolver size
// class, the item count and largest n (what decides the launches).
static std::string tune_signature(wpcd_batch b, int mode) {
  std::string sig = mode == WPCD_MIXED ? "mixed" : "f64";
  char buf[64];
  for (int c = 0; c < kNumClasses; ++c) {
    snprintf(buf, sizeof(buf), ":%d/%d", b->class_ptr[c + 1] - b->class_ptr[c], b->class_maxn[c]);
    sig += buf;
  }
  return sig;
}

int wpcd_autotune(wpcd_batch b, const wpcd_path_args* a, int mode, int reps, const char* cache_path,
                  wpcd_tune_result* out, hipStream_t stream) {
  if (!b || !a || !out) return fail(WPCD_ERR_INVALID, "wpcd_autotune: NULL argument");
  if (reps < 1 || reps > 100) return fail(WPCD_ERR_INVALID, "wpcd_autotune: reps must be in [1, 100]");
  if (mode != WPCD_MIXED && mode != WPCD_F64) return fail(WPCD_ERR_INVALID, "wpcd_autotune: unknown mode %d", mode);
  memset(out, 0, sizeof(*out));
  wpcd_ctx ctx = b->ctx;
  const std::string sig = tune_signature(b, mode);
  // the tune cache: one line per signature, "<signature> <jacobi_block> <refine_gemm> <ms>"
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[512], key[400];
      int jb = 0, rg = 0;
      double ms = 0.0;
      bool hit = false;
      while (fgets(line, sizeof(line), f))
        if (sscanf(line, "%399s %d %d %lf", key, &jb, &rg, &ms) == 4 && sig == key && jb >= 0 && jb <= 6 &&
            (rg == 0 || rg == 1)) {
          out->jacobi_block = jb;
          out->refine_gemm = rg;
          out->best_ms = ms;
          hit = true;  // the last matching line wins
        }
      fclose(f);
      if (hit) {
        out->from_cache = 1;
        ctx->cfg.jacobi_block = out->jacobi_block;
        ctx->cfg.refine_gemm = out->refine_gemm;
        return WPCD_OK;
      }
    }
  }
  if (ctx->profiling) return fail(WPCD_ERR_INVALID, "wpcd_autotune: the stage timers are on");
  WPCD_HIPX(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  WPCD_STICKY(ctx);
  // candidates: LDS Jacobi variant (two-column blocks / four-column blocks
  // with one angle per quarter row) x refinement products (whole-item /
  // tiles); the FP64 path has one schedule
  const int cand[4][2] = {{0, 0}, {5, 0}, {0, 1}, {5, 1}};
  const int n_cand = mode == WPCD_MIXED ? 4 : 1;
  const wpcd_config saved = ctx->cfg;
  // the runs go to the caller's stream, in order after the work already
  // there (they use the batch's work-space)
  hipStream_t st = stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = e == hipSuccess ? WPCD_OK : hip_fail(e, "wpcd_autotune: events");
  double best = 0.0;
  int best_i = 0;
  for (int i = 0; i < n_cand && rc == WPCD_OK; ++i) {
    ctx->cfg.jacobi_block = cand[i][0];
    ctx->cfg.refine_gemm = cand[i][1];
    rc = wpcd_run(b, a, mode, st);  // warm-up (first use of kernels and streams)
    if (rc == WPCD_OK) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && rc == WPCD_OK && e == hipSuccess; ++r) rc = wpcd_run(b, a, mode, st);
    if (rc == WPCD_OK && e == hipSuccess) e = hipEventRecord(e1, st);
    if (rc == WPCD_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (rc == WPCD_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (rc == WPCD_OK && e != hipSuccess) rc = dev_fail(ctx, e, "wpcd_autotune: timing");
    if (rc != WPCD_OK) break;
    out->cand_ms[i] = (double)ms / reps;
    if (i == 0 || out->cand_ms[i] < best) {
      best = out->cand_ms[i];
      best_i = i;
    }
  }
  if (e1) hipEventDestroy(e1);
  if (e0) hipEventDestroy(e0);
  ctx->cfg = saved;
  if (rc != WPCD_OK) return rc;
  out->n_cand = n_cand;
  out->jacobi_block = mode == WPCD_MIXED ? cand[best_i][0] : saved.jacobi_block;
  out->refine_gemm = mode == WPCD_MIXED ? cand[best_i][1] : saved.refine_gemm;
  out->best_ms = best;
  ctx->cfg.jacobi_block = out->jacobi_block;
  ctx->cfg.refine_gemm = out->refine_gemm;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(WPCD_ERR_INVALID, "wpcd_autotune: cannot append to the tune cache %s", cache_path);
    fprintf(f, "%s %d %d %.6f\n", sig.c_str(), out->jacobi_block, out->refine_gemm, best);
    fclose(f);
  }
  return WPCD_OK;
}

}  // extern "C"

struct wpcd_graph_s {
  wpcd_ctx ctx = nullptr;
  int device = 0;  // the context's device (destroy must not read the context: it may be gone)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t nodes = 0;
};

extern "C" {

int wpcd_graph_create(wpcd_batch b, const wpcd_path_args* a, int mode, wpcd_graph* out) {
  if (!b || !a || !out) return fail(WPCD_ERR_INVALID, "wpcd_graph_create: NULL argument");
  *out = nullptr;
  if (b->ctx->profiling)
    return fail(WPCD_ERR_INVALID, "wpcd_graph_create: the stage timers are on (they cannot time a graph's replays)");
  WPCD_HIPX(b->ctx, hipSetDevice(b->ctx->device), "hipSetDevice");
  WPCD_STICKY(b->ctx);
  if (mode == WPCD_MIXED) {
    const int rc = ensure_side(b->ctx);  // before the capture: the capture creates no stream
    if (rc != WPCD_OK) return rc;
  }
  hipStream_t cs = nullptr;
  WPCD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "wpcd_graph_create: capture stream");
  wpcd_graph_s* g = new (std::nothrow) wpcd_graph_s;
  if (!g) {
    hipStreamDestroy(cs);
    return fail(WPCD_ERR_NOMEM, "wpcd_graph_create: host allocation");
  }
  g->ctx = b->ctx;
  g->device = b->ctx->device;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = e == hipSuccess ? wpcd_run(b, a, mode, cs) : WPCD_OK;
  std::string run_err = rc != WPCD_OK ? g_err : std::string();
  // end the capture in every case (a failed run leaves a partial graph)
  hipGraph_t graph = nullptr;
  const hipError_t e_end = e == hipSuccess ? hipStreamEndCapture(cs, &graph) : e;
  if (rc == WPCD_OK && e_end == hipSuccess && graph) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  else if (e == hipSuccess) e = e_end;
  g->graph = graph;
  if (e == hipSuccess && graph) e = hipGraphGetNodes(graph, nullptr, &g->nodes);
  hipStreamDestroy(cs);
  if (rc != WPCD_OK || e != hipSuccess || !g->exec) {
    wpcd_graph_destroy(g);
    if (rc != WPCD_OK) return fail(rc, "wpcd_graph_create: %s", run_err.c_str());
    return hip_fail(e != hipSuccess ? e : hipErrorUnknown, "wpcd_graph_create: capture");
  }
  *out = g;
  return WPCD_OK;
}

int wpcd_graph_launch(wpcd_graph g, hipStream_t stream) {
  if (!g) return fail(WPCD_ERR_INVALID, "wpcd_graph_launch: NULL graph");
  WPCD_HIPX(g->ctx, hipSetDevice(g->ctx->device), "hipSetDevice");
  WPCD_STICKY(g->ctx);
  WPCD_HIPX(g->ctx, hipGraphLaunch(g->exec, stream), "wpcd_graph_launch");
  return WPCD_OK;
}

int wpcd_graph_nodes(wpcd_graph g, int64_t* nodes) {
  if (!g || !nodes) return fail(WPCD_ERR_INVALID, "wpcd_graph_nodes: NULL argument");
  *nodes = (int64_t)g->nodes;
  return WPCD_OK;
}

void wpcd_graph_destroy(wpcd_graph g) {
  if (!g) return;
  hipSetDevice(g->device);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

int wpcd_profile_enable(wpcd_ctx ctx, int on) {
  if (!ctx) return fail(WPCD_ERR_INVALID, "wpcd_profile_enable: NULL context");
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  for (auto& p : ctx->pending) {
    hipEventSynchronize(p.stop);
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->pending.clear();
  for (int i = 0; i < WPCD_N_STAGES; ++i) {
    ctx->stage_ms[i] = 0.0;
    ctx->stage_launches[i] = 0;
  }
  WPCD_HIP(hipMemset(ctx->d_counters, 0, 4 * sizeof(unsigned long long)), "wpcd_profile_enable: counters");
  ctx->profiling = on != 0;
  return WPCD_OK;
}

int wpcd_jacobi_counts(wpcd_ctx ctx, int64_t* counts_host) {
  if (!ctx || !counts_host) return fail(WPCD_ERR_INVALID, "wpcd_jacobi_counts: NULL argument");
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  WPCD_HIP(hipDeviceSynchronize(), "wpcd_jacobi_counts: synchronise");
  unsigned long long h[4];
  WPCD_HIP(hipMemcpy(h, ctx->d_counters, sizeof(h), hipMemcpyDeviceToHost), "wpcd_jacobi_counts: copy");
  for (int i = 0; i < 3; ++i) counts_host[i] = (int64_t)h[i];
  return WPCD_OK;
}

int wpcd_batch_jacobi_launches(wpcd_batch b, int clear, int64_t* counts_host) {
  if (!b || !counts_host) return fail(WPCD_ERR_INVALID, "wpcd_batch_jacobi_launches: NULL argument");
  counts_host[0] = b->jfb.launches;
  counts_host[1] = b->jfb.sweeps;
  if (clear) b->jfb.launches = b->jfb.sweeps = 0;
  return WPCD_OK;
}

int wpcd_stage_times(wpcd_ctx ctx, double* ms_host, int64_t* launches_host) {
  if (!ctx) return fail(WPCD_ERR_INVALID, "wpcd_stage_times: NULL context");
  WPCD_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipError_t err = hipSuccess;
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e == hipSuccess) {
      ctx->stage_ms[p.stage] += ms;
      ctx->stage_launches[p.stage] += 1;
    } else if (err == hipSuccess) {
      err = e;
    }
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->pending.clear();
  if (err != hipSuccess) return hip_fail(err, "wpcd_stage_times");
  for (int i = 0; i < WPCD_N_STAGES; ++i) {
    if (ms_host) ms_host[i] = ctx->stage_ms[i];
    if (launches_host) launches_host[i] = ctx->stage_launches[i];
  }
  return WPCD_OK;
}

}  // extern "C"
