// Request loop with continuous batching (the wpcd_server_* / wpcd_submit /
// wpcd_poll part of the C ABI).  Host code only: the worker thread packs
// admitted requests into one batch inside a device arena and drives the same
// kernel launchers as the batch API on one stream per in-flight slot.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "handles.h"
#include "internal.h"

using namespace wpcd;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct ReqChannel {
  int basis, grid, nch, N, n, J, n_terms;
};

enum { kQueued = 0, kRunning = 1, kDone = 2 };

struct Req {
  uint64_t ticket = 0;
  std::vector<ReqChannel> ch;
  std::vector<double> coef;  // concatenated per channel
  std::vector<double> tlab;
  double* sigma_host = nullptr;
  double* delta_host = nullptr;
  double* mix_host = nullptr;
  int32_t* status_host = nullptr;
  size_t bytes = 0;  // device footprint bound
  int state = kQueued;
  int code = WPCD_OK;
};

// Per-item and per-request device bytes (each array is padded to kAlign once
// per batch, accounted for separately).
size_t item_bytes(const ReqChannel& c) {
  const size_t n = c.n, N = c.N, K = c.nch;
  return sizeof(ItemDev) + 3 * sizeof(int32_t) + 8 * c.n_terms +              // descriptors, class, sitems, coef
         n * n * (8 + 8 + 4) + 8 * eig_work_doubles((int)n) +                // v64, evec, x32, work
         n * (4 + 8 + 8) +                                                    // cl, lam, eval
         8 * (2 * N * K * K + N * K + N + N * K) + 2 * sizeof(int32_t);      // t, delta, mix, s_dev, statuses
}
constexpr int kBatchArrays = 24;

// Offsets of one batch's arrays inside its arena block.
struct Layout {
  // upload region
  size_t items, cls, sptr, sitems, coef, tlab, toff, up_end;
  // download region
  size_t est, tst, sigma, delta, mix, down_end;
  // device-only
  size_t v64, evec, x32, work, cl, lam, eval, t, sdev, total;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  bool busy = false;
  size_t arena_off = 0, arena_bytes = 0;
  Layout L{};
  std::vector<Req*> reqs;
  std::vector<int64_t> d_off, m_off;  // per item delta / mix offsets
  int64_t n_items = 0;
  hipError_t err = hipSuccess;
  // launch counters of the device-memory Jacobi of this slot's batches; no
  // pinned flags, so every sweep is enqueued: the worker thread must not wait
  // on the device while requests arrive
  wpcd::JacFeedback jfb;
};

}  // namespace

struct wpcd_server_s {
  wpcd_ctx ctx = nullptr;
  int device = 0;  // the context's device (destroy must not read the context: it may be gone)
  wpcd_server_config cfg{};
  std::vector<GridHost*> grids_host;
  std::vector<BasisHost> bases;
  GridDev* d_grids = nullptr;
  BasisDev* d_bases = nullptr;
  char* arena_mem = nullptr;
  wpcd::Arena arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  wpcd_server_stats st{};

  void run();
  bool launch(Slot& s, std::vector<Req*>& take);
  void finish(Slot& s);
};

namespace {

int sfail(int code, const char* msg) { return set_error(code, msg); }

Layout plan(const std::vector<Req*>& take, int64_t& n_items) {
  Layout L{};
  int64_t ni = 0, nc = 0, nt = 0, vv = 0, ne = 0, td = 0, de = 0, me = 0, wd = 0;
  for (Req* r : take) {
    nt += r->tlab.size();
    for (auto& c : r->ch) {
      ni++;
      nc += c.n_terms;
      vv += (int64_t)c.n * c.n;
      wd += eig_work_doubles(c.n);
      ne += c.n;
      td += 2LL * c.N * c.nch * c.nch;
      de += (int64_t)c.N * c.nch;
      me += c.N;
    }
  }
  const int64_t nr = (int64_t)take.size();
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.items = put(sizeof(ItemDev) * ni);
  L.cls = put(4 * ni);
  L.sptr = put(4 * (nr + 1));
  L.sitems = put(4 * ni);
  L.coef = put(8 * std::max<int64_t>(nc, 1));
  L.tlab = put(8 * std::max<int64_t>(nt, 1));
  L.toff = put(4 * (nr + 1));
  L.up_end = o;
  L.est = put(4 * ni);
  L.tst = put(4 * ni);
  L.sigma = put(8 * std::max<int64_t>(nt, 1));
  L.delta = put(8 * de);
  L.mix = put(8 * me);
  L.down_end = o;
  L.v64 = put(8 * vv);
  L.evec = put(8 * vv);
  L.x32 = put(4 * vv);
  L.work = put(8 * wd);
  L.cl = put(4 * ne);
  L.lam = put(8 * ne);
  L.eval = put(8 * ne);
  L.t = put(8 * td);
  L.sdev = put(8 * de);
  L.total = o;
  n_items = ni;
  return L;
}

}  // namespace

bool wpcd_server_s::launch(Slot& s, std::vector<Req*>& take) {
  int64_t ni = 0;
  const Layout L = plan(take, ni);
  const size_t off = arena.alloc(L.total);
  if (off == SIZE_MAX) return false;
  s.arena_off = off;
  s.arena_bytes = L.total;
  s.L = L;
  s.n_items = ni;
  s.reqs = take;
  s.err = hipSuccess;
  const size_t pin_need = L.up_end + (L.down_end - L.est);
  if (s.pinned_bytes < pin_need) {
    if (s.pinned) hipHostFree(s.pinned);
    s.pinned = nullptr;
    s.pinned_bytes = 0;
    const size_t want = std::max(pin_need, (size_t)1 << 20) * 2;
    if (hipHostMalloc((void**)&s.pinned, want, hipHostMallocDefault) != hipSuccess) {
      s.pinned = nullptr;
      s.err = hipErrorOutOfMemory;
    } else {
      s.pinned_bytes = want;
    }
  }
  // host-side descriptors straight into the pinned upload region
  s.d_off.assign(ni, 0);
  s.m_off.assign(ni, 0);
  int class_ptr[kNumClasses + 1] = {0}, class_maxn[kNumClasses] = {0};
  int max_n = 0, min_n = 0, max_nbins = 0;
  if (s.err == hipSuccess) {
    char* P = s.pinned;
    ItemDev* items = reinterpret_cast<ItemDev*>(P + L.items);
    int32_t* cls = reinterpret_cast<int32_t*>(P + L.cls);
    int32_t* sptr = reinterpret_cast<int32_t*>(P + L.sptr);
    int32_t* sitems = reinterpret_cast<int32_t*>(P + L.sitems);
    double* coef = reinterpret_cast<double*>(P + L.coef);
    double* tlab = reinterpret_cast<double*>(P + L.tlab);
    int32_t* toff = reinterpret_cast<int32_t*>(P + L.toff);
    int64_t i = 0, v = 0, e = 0, t = 0, d = 0, m = 0, c = 0, w = 0;
    int32_t tj = 0;
    for (size_t r = 0; r < take.size(); ++r) {
      Req* q = take[r];
      sptr[r] = (int32_t)i;
      toff[r] = tj;
      std::copy(q->tlab.begin(), q->tlab.end(), tlab + tj);
      tj += (int32_t)q->tlab.size();
      size_t cc = 0;
      for (auto& ch : q->ch) {
        ItemDev& it = items[i];
        memset(&it, 0, sizeof(it));
        it.grid = ch.grid;
        it.nch = ch.nch;
        it.N = ch.N;
        it.n = ch.n;
        it.ng = grids_host[ch.grid]->ng;
        it.J = ch.J;
        it.sample = (int32_t)r;
        it.basis = ch.basis;
        it.spin = -1;
        it.l0 = -1;
        it.u_off = 0;
        it.v_off = v;
        it.e_off = e;
        it.t_off = t;
        it.d_off = d;
        it.m_off = m;
        it.w_off = w;
        it.c_off = c;
        std::copy(q->coef.begin() + cc, q->coef.begin() + cc + ch.n_terms, coef + c);
        cc += ch.n_terms;
        s.d_off[i] = d;
        s.m_off[i] = m;
        sitems[i] = (int32_t)i;
        v += (int64_t)ch.n * ch.n;
        e += ch.n;
        t += 2LL * ch.N * ch.nch * ch.nch;
        d += (int64_t)ch.N * ch.nch;
        m += ch.N;
        c += ch.n_terms;
        w += eig_work_doubles(ch.n);
        max_n = std::max(max_n, ch.n);
        min_n = min_n == 0 ? ch.n : std::min(min_n, ch.n);
        max_nbins = std::max(max_nbins, ch.N);
        class_ptr[size_class(ch.n) + 1]++;
        class_maxn[size_class(ch.n)] = std::max(class_maxn[size_class(ch.n)], ch.n);
        ++i;
      }
    }
    sptr[take.size()] = (int32_t)i;
    toff[take.size()] = tj;
    for (int k = 0; k < kNumClasses; ++k) class_ptr[k + 1] += class_ptr[k];
    int fill[kNumClasses];
    for (int k = 0; k < kNumClasses; ++k) fill[k] = class_ptr[k];
    for (int64_t j = 0; j < ni; ++j) cls[fill[size_class(items[j].n)]++] = (int32_t)j;
  }
  // device pointers
  char* D = arena_mem + off;
  auto dp = [&](size_t o) { return D + o; };
  const ItemDev* d_items = reinterpret_cast<const ItemDev*>(dp(L.items));
  const int32_t* d_cls = reinterpret_cast<const int32_t*>(dp(L.cls));
  const int32_t* d_sptr = reinterpret_cast<const int32_t*>(dp(L.sptr));
  const int32_t* d_sitems = reinterpret_cast<const int32_t*>(dp(L.sitems));
  const double* d_coef = reinterpret_cast<const double*>(dp(L.coef));
  const double* d_tlab = reinterpret_cast<const double*>(dp(L.tlab));
  const int32_t* d_toff = reinterpret_cast<const int32_t*>(dp(L.toff));
  int32_t* d_est = reinterpret_cast<int32_t*>(dp(L.est));
  int32_t* d_tst = reinterpret_cast<int32_t*>(dp(L.tst));
  double* d_sigma = reinterpret_cast<double*>(dp(L.sigma));
  double* d_delta = reinterpret_cast<double*>(dp(L.delta));
  double* d_mix = reinterpret_cast<double*>(dp(L.mix));
  double* d_v64 = reinterpret_cast<double*>(dp(L.v64));
  double* d_evec = reinterpret_cast<double*>(dp(L.evec));
  float* d_x32 = reinterpret_cast<float*>(dp(L.x32));
  double* d_work = reinterpret_cast<double*>(dp(L.work));
  int32_t* d_cl = reinterpret_cast<int32_t*>(dp(L.cl));
  double* d_lam = reinterpret_cast<double*>(dp(L.lam));
  double* d_eval = reinterpret_cast<double*>(dp(L.eval));
  double* d_t = reinterpret_cast<double*>(dp(L.t));
  double* d_sdev = reinterpret_cast<double*>(dp(L.sdev));
  const wpcd_config& c = ctx->cfg;
  hipError_t e = s.err;
  const int n = (int)ni;
  if (e == hipSuccess) e = hipMemcpyAsync(D, s.pinned, L.up_end, hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess) e = launch_project_affine(d_items, n, max_n, d_bases, d_coef, d_v64, s.stream);
  for (int k = 0; k < kNumClasses && e == hipSuccess; ++k) {
    const int n_sel = class_ptr[k + 1] - class_ptr[k];
    if (n_sel == 0) continue;
    if (k < kNumClasses - 1)
      e = launch_jacobi_f32_lds(d_items, d_cls + class_ptr[k], n_sel, class_maxn[k], d_grids, d_v64, d_x32, d_eval,
                                d_est, c.max_sweeps, (float)c.jacobi_tol_f32, (float)c.jacobi_stop_f32, c.jacobi_block,
                                nullptr, d_work, nullptr, s.stream);
    else
      e = launch_jacobi_global(1, d_items, d_cls + class_ptr[k], n_sel, class_maxn[k], d_grids, d_v64, d_work,
                               d_evec, d_x32, d_eval, d_est, c.max_sweeps, c.jacobi_tol_f32, c.jacobi_stop_f32,
                               nullptr, &s.jfb, s.stream);
  }
  if (e == hipSuccess)
    e = launch_refine(d_items, n, min_n, max_n, d_grids, d_v64, d_x32, d_evec, d_eval, d_lam, d_work, d_cl, d_est,
                      std::max(1, c.refine_steps), c.refine_close_log10, c.refine_gemm, c.refine_rr_steps, s.stream, nullptr,
                      nullptr,
                      nullptr);
  if (e == hipSuccess)
    e = launch_tmatrix(d_items, n, max_n, d_grids, d_v64, d_eval, d_evec, WPCD_MIXED, d_t, d_tst, s.stream);
  if (e == hipSuccess) e = launch_observables(d_items, n, max_nbins, d_grids, d_t, d_delta, d_mix, d_sdev, s.stream);
  if (e == hipSuccess)
    e = launch_sigma(d_items, d_sptr, d_sitems, (int)take.size(), d_grids, d_delta, d_mix, d_tlab, d_toff, 0,
                     d_sigma, s.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.pinned + L.up_end, dp(L.est), L.down_end - L.est, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
  s.err = e;
  s.busy = true;
  {
    std::lock_guard<std::mutex> lk(mu);
    st.batches++;
    st.items += ni;
    st.jacobi_launches += s.jfb.launches;
    st.jacobi_sweeps += s.jfb.sweeps;
    s.jfb.launches = s.jfb.sweeps = 0;
    st.peak_arena_bytes = std::max<int64_t>(st.peak_arena_bytes, (int64_t)arena.used());
  }
  return true;
}

void wpcd_server_s::finish(Slot& s) {
  const Layout& L = s.L;
  const char* H = s.pinned + L.up_end;  // download region, based at L.est
  const int32_t* est = reinterpret_cast<const int32_t*>(H + (L.est - L.est));
  const int32_t* tst = reinterpret_cast<const int32_t*>(H + (L.tst - L.est));
  const double* sigma = reinterpret_cast<const double*>(H + (L.sigma - L.est));
  const double* delta = reinterpret_cast<const double*>(H + (L.delta - L.est));
  const double* mix = reinterpret_cast<const double*>(H + (L.mix - L.est));
  int64_t i = 0, tj = 0;
  for (Req* q : s.reqs) {
    int code = WPCD_OK;
    if (s.err != hipSuccess) {
      code = WPCD_ERR_DEVICE;
    } else {
      if (q->sigma_host) std::copy(sigma + tj, sigma + tj + q->tlab.size(), q->sigma_host);
      int64_t dd = 0, mm = 0;
      for (size_t k = 0; k < q->ch.size(); ++k, ++i) {
        const ReqChannel& ch = q->ch[k];
        int32_t sc = est[i] <= 0 ? est[i] : (tst[i] != 0 ? tst[i] : est[i]);
        if (sc <= 0 && code == WPCD_OK) code = sc;
        if (q->status_host) q->status_host[k] = sc;
        const int64_t nd = (int64_t)ch.N * ch.nch;
        if (q->delta_host) std::copy(delta + s.d_off[i], delta + s.d_off[i] + nd, q->delta_host + dd);
        if (q->mix_host) std::copy(mix + s.m_off[i], mix + s.m_off[i] + ch.N, q->mix_host + mm);
        dd += nd;
        mm += ch.N;
      }
    }
    tj += q->tlab.size();
    q->code = code;
  }
  arena.release(s.arena_off, s.arena_bytes);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Req* q : s.reqs) q->state = kDone;
    st.completed += (int64_t)s.reqs.size();
    st.inflight--;
  }
  cv.notify_all();
  s.reqs.clear();
  s.busy = false;
}

void wpcd_server_s::run() {
  hipSetDevice(ctx->device);
  std::vector<Req*> take;
  for (;;) {
    bool progressed = false;
    // completions
    for (Slot& s : slots) {
      if (!s.busy) continue;
      hipError_t q = s.err != hipSuccess ? hipSuccess : hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess && s.err == hipSuccess) s.err = q;
      if (s.err != hipSuccess) hipStreamSynchronize(s.stream);  // drain what was enqueued
      finish(s);
      progressed = true;
    }
    // admission: arrival order, while the footprint fits one arena block
    Slot* free_slot = nullptr;
    for (Slot& s : slots)
      if (!s.busy) {
        free_slot = &s;
        break;
      }
    bool stopping = false;
    if (free_slot) {
      take.clear();
      {
        std::lock_guard<std::mutex> lk(mu);
        stopping = stop;
        if (!stop) {
          const size_t room = arena.largest();
          size_t bytes = kBatchArrays * kAlign;
          int64_t items = 0;
          while (!queue.empty()) {
            Req* r = queue.front();
            if (!take.empty() && items + (int64_t)r->ch.size() > cfg.max_batch_items) break;
            if (bytes + r->bytes > room) break;
            bytes += r->bytes;
            items += (int64_t)r->ch.size();
            take.push_back(r);
            r->state = kRunning;
            queue.pop_front();
          }
          st.queued = (int32_t)queue.size();
          if (!take.empty()) st.inflight++;
        }
      }
      if (!take.empty()) {
        if (!launch(*free_slot, take)) {
          // cannot happen (the block was measured under the same thread); requeue
          std::lock_guard<std::mutex> lk(mu);
          for (auto it = take.rbegin(); it != take.rend(); ++it) {
            (*it)->state = kQueued;
            queue.push_front(*it);
          }
          st.inflight--;
        }
        progressed = true;
      }
    } else {
      std::lock_guard<std::mutex> lk(mu);
      stopping = stop;
    }
    bool any_busy = false;
    for (Slot& s : slots) any_busy = any_busy || s.busy;
    if (stopping && !any_busy) break;
    if (progressed) continue;
    std::unique_lock<std::mutex> lk(mu);
    if (any_busy)
      cv.wait_for(lk, std::chrono::microseconds(20));
    else
      cv.wait(lk, [&] { return stop || !queue.empty(); });
  }
}

extern "C" {

int wpcd_server_create(wpcd_ctx ctx, const wpcd_server_config* cfg, wpcd_server* out) {
  if (!ctx || !out) return sfail(WPCD_ERR_INVALID, "wpcd_server_create: NULL argument");
  *out = nullptr;
  wpcd_server_config c{(int64_t)4 << 30, 4, 4096, 65536, 0};
  if (cfg) c = *cfg;
  if (c.hbm_budget_bytes < ((int64_t)1 << 20) || c.max_inflight < 1 || c.max_inflight > 8 ||
      c.max_batch_items < 1 || c.max_queue < 1)
    return sfail(WPCD_ERR_INVALID, "wpcd_server_create: bad configuration");
  if (hipSetDevice(ctx->device) != hipSuccess) return sfail(WPCD_ERR_DEVICE, "hipSetDevice failed");
  wpcd_server_s* s = new (std::nothrow) wpcd_server_s;
  if (!s) return sfail(WPCD_ERR_NOMEM, "wpcd_server_create: host allocation");
  s->ctx = ctx;
  s->device = ctx->device;
  s->cfg = c;
  s->bases = ctx->bases;
  for (auto& g : ctx->grids) s->grids_host.push_back(&g);
  std::vector<GridDev> gd;
  for (auto& g : ctx->grids) gd.push_back(g.dev);
  std::vector<BasisDev> bd;
  for (auto& b : ctx->bases) bd.push_back(BasisDev{b.dbuf, b.n, b.n_terms});
  hipError_t e = hipSuccess;
  if (!gd.empty()) e = hipMalloc((void**)&s->d_grids, sizeof(GridDev) * gd.size());
  if (e == hipSuccess && !gd.empty())
    e = hipMemcpy(s->d_grids, gd.data(), sizeof(GridDev) * gd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !bd.empty()) e = hipMalloc((void**)&s->d_bases, sizeof(BasisDev) * bd.size());
  if (e == hipSuccess && !bd.empty())
    e = hipMemcpy(s->d_bases, bd.data(), sizeof(BasisDev) * bd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&s->arena_mem, (size_t)c.hbm_budget_bytes);
  s->arena.reset((size_t)c.hbm_budget_bytes);
  s->slots.resize(c.max_inflight);
  for (auto& sl : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    wpcd_server_destroy(s);
    const std::string msg = std::string("wpcd_server_create: ") + hipGetErrorString(e);
    return sfail(e == hipErrorOutOfMemory ? WPCD_ERR_NOMEM : WPCD_ERR_DEVICE, msg.c_str());
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return WPCD_OK;
}

void wpcd_server_destroy(wpcd_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.pinned) hipHostFree(sl.pinned);
  }
  hipFree(s->arena_mem);
  hipFree(s->d_grids);
  hipFree(s->d_bases);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
}

int wpcd_submit(wpcd_server s, const wpcd_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return sfail(WPCD_ERR_INVALID, "wpcd_submit: NULL argument");
  if (req->n_channels < 1 || req->n_channels > 64 || !req->channels_host)
    return sfail(WPCD_ERR_INVALID, "wpcd_submit: need 1..64 channels");
  if (req->n_tlab < 0 || req->n_tlab > 1024 || (req->n_tlab > 0 && (!req->tlab_host || !req->sigma_host)))
    return sfail(WPCD_ERR_INVALID, "wpcd_submit: need 0..1024 T_lab values and a sigma buffer");
  Req* r = new (std::nothrow) Req;
  if (!r) return sfail(WPCD_ERR_NOMEM, "wpcd_submit: host allocation");
  r->ch.reserve(req->n_channels);
  size_t bytes = sizeof(int32_t) * 2 + 16 * (size_t)req->n_tlab;
  for (int k = 0; k < req->n_channels; ++k) {
    const wpcd_req_channel& in = req->channels_host[k];
    if (in.basis_id < 0 || in.basis_id >= (int)s->bases.size() || !in.coef_host) {
      delete r;
      return sfail(WPCD_ERR_INVALID, "wpcd_submit: unknown basis id or NULL coefficients");
    }
    const BasisHost& b = s->bases[in.basis_id];
    if (in.J < 0 || (b.nch == 2 && in.J < 1)) {
      delete r;
      return sfail(WPCD_ERR_INVALID, "wpcd_submit: need J >= 0 (>= 1 if coupled)");
    }
    ReqChannel c{in.basis_id, b.grid, b.nch, s->grids_host[b.grid]->N, b.n, in.J, b.n_terms};
    r->ch.push_back(c);
    r->coef.insert(r->coef.end(), in.coef_host, in.coef_host + b.n_terms);
    bytes += item_bytes(c);
  }
  if (req->n_tlab > 0) r->tlab.assign(req->tlab_host, req->tlab_host + req->n_tlab);
  r->sigma_host = req->sigma_host;
  r->delta_host = req->delta_host;
  r->mix_host = req->mix_host;
  r->status_host = req->status_host;
  r->bytes = bytes;
  if (bytes + kBatchArrays * kAlign > (size_t)s->cfg.hbm_budget_bytes) {
    delete r;
    return sfail(WPCD_ERR_UNSUPPORTED, "wpcd_submit: request exceeds the server's device budget");
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return sfail(WPCD_ERR_INVALID, "wpcd_submit: server is stopping");
    }
    if ((int64_t)s->queue.size() >= s->cfg.max_queue) {
      delete r;
      return sfail(WPCD_ERR_BUSY, "wpcd_submit: queue full");
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    s->st.submitted++;
    s->st.queued = (int32_t)s->queue.size();
    *ticket = r->ticket;
  }
  s->cv.notify_all();
  return WPCD_OK;
}

int wpcd_poll(wpcd_server s, uint64_t ticket) {
  if (!s) return sfail(WPCD_ERR_INVALID, "wpcd_poll: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(WPCD_ERR_INVALID, "wpcd_poll: unknown or retired ticket");
  Req* r = it->second;
  if (r->state != kDone) return WPCD_ERR_AGAIN;
  const int code = r->code;
  s->reqs.erase(it);
  delete r;
  if (code != WPCD_OK) sfail(code, "wpcd_poll: the request's batch or one of its items failed");
  return code;
}

int wpcd_server_stats_get(wpcd_server s, wpcd_server_stats* out) {
  if (!s || !out) return sfail(WPCD_ERR_INVALID, "wpcd_server_stats_get: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return WPCD_OK;
}

}  // extern "C"
