// C ABI of the library (declared in include/plsqr.h): engine lifetime, operator
// registration, request submission/completion, HBM-budget admission.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "engine.hpp"

using namespace plsqr;

namespace {

thread_local std::string g_last_error = "no error";

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(PLSQR_E_HIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hipGetDevice(&prev);
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    hipGetDevice(&cur);
    if (prev >= 0 && cur != prev) hipSetDevice(prev);
  }
};

// Fill the descriptor of request r (host copy) from its workspace layout.
void fill_desc(plsqr_engine *eng, Request &r, const Operator &op) {
  const Layout &Ly = r.lay;
  const plsqr_problem &pb = r.pb;
  char *ws = r.ws;
  InstDesc &D = r.host;
  std::memset(&D, 0, sizeof(D));
  D.nx = pb.nx;
  D.ny = pb.ny;
  D.nz = pb.nz;
  D.levels = Ly.levels;
  D.n = Ly.n;
  D.m = Ly.m;
  D.reg = pb.reg;
  D.op_kind = op.op.kind;
  D.radius = op.op.kind == PLSQR_OP_BLUR ? op.op.radius : 0;
  D.smoother = pb.smoother;
  D.nu_pre = pb.nu_pre;
  D.nu_post = pb.nu_post;
  D.cheb_degree = pb.cheb_degree;
  D.dims = pb.nz > 1 ? 3 : 2;
  D.T = (float)(pb.reg == PLSQR_REG_TIKHONOV ? 1.0 : pb.T);
  D.omega = (float)pb.omega;
  D.tau = pb.tau;
  D.eps = pb.eps;
  if (pb.smoother == PLSQR_SMOOTH_CHEBYSHEV) {
    D.cheb_theta = 0.5 * (pb.cheb_hi + pb.cheb_lo);
    D.cheb_delta = 0.5 * (pb.cheb_hi - pb.cheb_lo);
    D.cheb_sigma = D.cheb_theta / D.cheb_delta;
  }
  if (op.op.kind == PLSQR_OP_BLUR)
    for (size_t i = 0; i < op.taps.size() && i < (size_t)kMaxTaps; ++i) D.taps[i] = op.taps[i];
  D.g = r.g;
  D.A = op.op.kind == PLSQR_OP_DENSE ? op.op.A_dev : nullptr;
  auto F = [&](size_t off) { return reinterpret_cast<float *>(ws + off); };
  D.f = F(Ly.f);
  D.u = F(Ly.u);
  D.p = F(Ly.p);
  D.v = F(Ly.v);
  D.w = F(Ly.w);
  D.kappa = F(Ly.kappa);
  D.tmp1 = Ly.tmp1 ? F(Ly.tmp1) : nullptr;
  D.tmp2 = Ly.tmp2 ? F(Ly.tmp2) : nullptr;
  D.colpart = Ly.colpart ? F(Ly.colpart) : nullptr;
  D.colchunks = Ly.colchunks;
  D.out_f = r.f_out;
  D.sc = reinterpret_cast<double *>(ws + Ly.sc);
  D.part = reinterpret_cast<double *>(ws + Ly.part);
  D.cfac = reinterpret_cast<double *>(ws + Ly.cfac);
  D.diag = reinterpret_cast<double *>(ws + Ly.diag);
  D.nc = Ly.nc;
  const int d = pb.nz > 1 ? 3 : 2;
  for (int l = 0; l < Ly.levels; ++l) {
    LevelDesc &L = D.lv[l];
    L.nx = Ly.lnx[l];
    L.ny = Ly.lny[l];
    L.nz = Ly.lnz[l];
    L.n = Ly.ln[l];
    L.x = l == 0 ? D.v : F(Ly.lvl[l][0]);
    L.b = l == 0 ? D.p : F(Ly.lvl[l][1]);
    L.r = F(Ly.lvl[l][2]);
    L.t = F(Ly.lvl[l][3]);
    L.s = F(Ly.lvl[l][4]);
    L.wx = l > 0 ? F(Ly.lvl[l][5]) : nullptr;
    L.wy = l > 0 ? F(Ly.lvl[l][6]) : nullptr;
    L.wz = (l > 0 && Ly.lvl[l][7]) ? F(Ly.lvl[l][7]) : nullptr;
    L.dinv = F(Ly.lvl[l][8]);
    L.eps = pb.eps * std::ldexp(1.0, d * l);   // Galerkin: P^T (eps I) P = 2^d eps I
  }
  (void)eng;
}

// Pinned staging layout: [InstDesc][descriptor pointer][scalars][per-outer records].
size_t pin_desc_ptr_off() { return (sizeof(InstDesc) + 255) / 256 * 256; }
size_t pin_sc_off() { return pin_desc_ptr_off() + 256; }
size_t pin_dg_off() { return pin_sc_off() + SC_COUNT * sizeof(double); }

void release(plsqr_engine *eng, Request &r) {
  if (r.ev_start) hipEventDestroy(r.ev_start);
  if (r.ev_end) hipEventDestroy(r.ev_end);
  r.ev_start = r.ev_end = nullptr;
  for (auto *lst : {&r.prod_events, &r.adj_events}) {
    for (auto &e : *lst) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
    lst->clear();
  }
  if (r.ws) {
    eng->pool.put(r.ws, r.lay.total);
    eng->used -= r.lay.total;
    r.ws = nullptr;
  }
  if (r.pinned) hipHostFree(r.pinned);
  r.pinned = nullptr;
}

// Allocate and enqueue a request (state QUEUED -> RUNNING). Caller holds the lock.
// Nothing here waits for earlier work on the stream: the descriptor goes up and the
// results come down through pinned host memory with stream-ordered copies.
int start_request_impl(plsqr_engine *eng, Request &r) {
  const Operator &op = eng->ops[r.op_id];
  r.ws = static_cast<char *>(eng->pool.get(r.lay.total));
  if (!r.ws) return set_error(PLSQR_E_NOMEM, "device allocation of the request workspace failed");
  eng->used += r.lay.total;
  r.pinned_bytes = pin_dg_off() + (size_t)(r.pb.outer + 1) * DG_COUNT * sizeof(double);
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&r.pinned), r.pinned_bytes, hipHostMallocDefault));
  fill_desc(eng, r, op);
  r.d_descs = reinterpret_cast<InstDesc **>(r.ws + r.lay.descptr);
  InstDesc *d_desc = reinterpret_cast<InstDesc *>(r.ws + r.lay.desc);
  std::memcpy(r.pinned, &r.host, sizeof(InstDesc));
  std::memcpy(r.pinned + pin_desc_ptr_off(), &d_desc, sizeof(void *));
  HIP_TRY(hipEventCreate(&r.ev_start));
  HIP_TRY(hipEventCreate(&r.ev_end));
  HIP_TRY(hipEventRecord(r.ev_start, eng->stream));
  HIP_TRY(hipMemcpyAsync(d_desc, r.pinned, sizeof(InstDesc), hipMemcpyHostToDevice, eng->stream));
  HIP_TRY(hipMemcpyAsync(r.d_descs, r.pinned + pin_desc_ptr_off(), sizeof(void *),
                         hipMemcpyHostToDevice, eng->stream));
  const bool timed = (r.pb.flags & PLSQR_FLAG_TIME_PRODUCTS) != 0;
  BatchView bv{r.d_descs, 1, &r.host, &r.lay, timed ? &r.prod_events : nullptr,
               timed ? &r.adj_events : nullptr};
  enqueue_whole_solve(eng->stream, bv, r.pb.outer, r.pb.inner);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(r.pinned + pin_sc_off(), r.ws + r.lay.sc, SC_COUNT * sizeof(double),
                         hipMemcpyDeviceToHost, eng->stream));
  HIP_TRY(hipMemcpyAsync(r.pinned + pin_dg_off(), r.ws + r.lay.diag,
                         (size_t)(r.pb.outer + 1) * DG_COUNT * sizeof(double),
                         hipMemcpyDeviceToHost, eng->stream));
  HIP_TRY(hipEventRecord(r.ev_end, eng->stream));
  r.state = Request::RUNNING;
  return PLSQR_OK;
}

int start_request(plsqr_engine *eng, Request &r) {
  const int rc = start_request_impl(eng, r);
  if (rc != PLSQR_OK) {
    hipStreamSynchronize(eng->stream);
    release(eng, r);
  }
  return rc;
}

// Collect a finished request: read diagnostics, release its memory.
void reap(plsqr_engine *eng, Request &r) {
  plsqr_result &res = r.result;
  std::memset(&res, 0, sizeof(res));
  const double *sc = reinterpret_cast<const double *>(r.pinned + pin_sc_off());
  const double *dg = reinterpret_cast<const double *>(r.pinned + pin_dg_off());
  res.status = (int)sc[SC_STATUS];
  res.outer_done = r.pb.outer;
  res.levels = r.lay.levels;
  for (int k = 1; k <= r.pb.outer; ++k) {
    res.resid[k - 1] = dg[(size_t)k * DG_COUNT + DG_RESID];
    res.penalty[k - 1] = dg[(size_t)k * DG_COUNT + DG_PENALTY];
    res.inner_done[k - 1] = (int)dg[(size_t)k * DG_COUNT + DG_INNER];
  }
  float ms = 0.f;
  if (r.ev_start && r.ev_end && hipEventElapsedTime(&ms, r.ev_start, r.ev_end) == hipSuccess)
    res.device_ms = ms;
  auto total = [](const std::vector<std::pair<hipEvent_t, hipEvent_t>> &lst) {
    double s = 0.0;
    for (auto &e : lst) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) s += t;
    }
    return s;
  };
  res.forward_ms = total(r.prod_events);
  res.forward_launches = (int64_t)r.prod_events.size();
  res.adjoint_ms = total(r.adj_events);
  res.adjoint_launches = (int64_t)r.adj_events.size();
  res.workspace_bytes = (int64_t)r.lay.total;
  r.t_done = now_ms();
  res.submit_to_done_ms = r.t_done - r.t_submit;
  release(eng, r);
  r.status = res.status;
  r.state = Request::DONE;
}

// Reap every finished running request, then start queued ones that now fit.
void progress(plsqr_engine *eng) {
  for (auto &kv : eng->reqs) {
    Request &r = *kv.second;
    if (r.state == Request::RUNNING && hipEventQuery(r.ev_end) == hipSuccess) reap(eng, r);
  }
  while (!eng->queued.empty()) {
    auto it = eng->reqs.find(eng->queued.front());
    if (it == eng->reqs.end()) {
      eng->queued.pop_front();
      continue;
    }
    Request &r = *it->second;
    if (eng->budget && eng->used + r.lay.total > eng->budget) break;
    eng->queued.pop_front();
    const int rc = start_request(eng, r);
    if (rc != PLSQR_OK) {
      r.status = rc;
      r.state = Request::DONE;
      std::memset(&r.result, 0, sizeof(r.result));
      r.result.status = rc;
    }
  }
}

}  // namespace

namespace plsqr {
Pool::~Pool() { trim(); }
void *Pool::get(size_t bytes) {
  auto it = free_.find(bytes);
  if (it != free_.end()) {
    void *p = it->second;
    free_.erase(it);
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    trim();
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  }
  return p;
}
void Pool::put(void *p, size_t bytes) { free_.emplace(bytes, p); }
void Pool::trim() {
  for (auto &kv : free_) hipFree(kv.second);
  free_.clear();
}
}  // namespace plsqr

extern "C" {

int plsqr_auto_levels(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  int levels = 1;
  long long a[3] = {nx, ny, nz};
  const int na = nz > 1 ? 3 : 2;
  while (levels < kMaxLevels) {
    bool ok = true;
    for (int i = 0; i < na; ++i) ok = ok && (a[i] % 2 == 0) && (a[i] > 4);
    if (!ok) break;
    for (int i = 0; i < na; ++i) a[i] /= 2;
    ++levels;
  }
  return levels;
}

uint64_t plsqr_workspace_bytes(const plsqr_problem *prob, int32_t op_kind, int64_t n_y) {
  if (!prob || n_y < 1) return 0;
  if (op_kind != PLSQR_OP_BLUR && op_kind != PLSQR_OP_DENSE) return 0;
  int levels = prob->mg_levels ? prob->mg_levels : plsqr_auto_levels(prob->nx, prob->ny, prob->nz);
  if (levels < 1 || levels > kMaxLevels) return 0;
  return make_layout(*prob, n_y, levels, op_kind).total;
}

int plsqr_create(plsqr_engine **out, int device, uint64_t hbm_budget_bytes, void *hip_stream,
                 uint32_t flags) {
  if (!out) return set_error(PLSQR_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return set_error(PLSQR_E_HIP, "no HIP device available");
  if (device < 0 || device >= ndev) return set_error(PLSQR_E_INVALID, "device index out of range");
  if (flags & ~(uint32_t)PLSQR_ENGINE_SERVE) return set_error(PLSQR_E_INVALID, "unknown engine flags");
  if (flags & PLSQR_ENGINE_SERVE)
    return set_error(PLSQR_E_INVALID, "serving mode is not available in this build");
  auto *e = new plsqr_engine();
  e->device = device;
  e->stream = static_cast<hipStream_t>(hip_stream);
  e->budget = hbm_budget_bytes;
  e->flags = flags;
  *out = e;
  return PLSQR_OK;
}

int plsqr_set_operator(plsqr_engine *eng, const plsqr_operator *op, int32_t *op_id) {
  if (!eng || !op || !op_id) return set_error(PLSQR_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(eng->mu);
  if (op->nx < 1 || op->ny < 1 || op->nz < 1) return set_error(PLSQR_E_INVALID, "bad operator grid");
  Operator o;
  o.op = *op;
  if (op->kind == PLSQR_OP_BLUR) {
    if (op->radius < 0 || op->radius > PLSQR_MAX_RADIUS)
      return set_error(PLSQR_E_INVALID, "blur radius out of range [0, 16]");
    if (!op->taps) return set_error(PLSQR_E_INVALID, "blur taps pointer is NULL");
    o.taps.assign(op->taps, op->taps + 2 * op->radius + 1);
    for (float t : o.taps)
      if (!std::isfinite(t)) return set_error(PLSQR_E_INVALID, "blur taps must be finite");
    o.op.taps = nullptr;
    o.op.n_y = (int64_t)op->nx * op->ny * op->nz;
    o.op.A_dev = nullptr;
    o.op.A_hi_dev = o.op.A_lo_dev = nullptr;
  } else if (op->kind == PLSQR_OP_DENSE) {
    if (op->n_y < 1) return set_error(PLSQR_E_INVALID, "dense operator needs n_y >= 1");
    if (!op->A_dev) return set_error(PLSQR_E_INVALID, "dense operator needs A_dev");
  } else {
    return set_error(PLSQR_E_INVALID, "unknown operator kind");
  }
  eng->ops.push_back(o);
  *op_id = (int32_t)eng->ops.size() - 1;
  return PLSQR_OK;
}

int plsqr_solve(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob, const float *g_dev,
                float *f_dev, uint64_t *ticket) {
  if (!eng || !prob || !ticket) return set_error(PLSQR_E_INVALID, "null argument");
  if (!g_dev || !f_dev) return set_error(PLSQR_E_INVALID, "g_dev and f_dev must be device pointers");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  const Operator *op = (op_id >= 0 && op_id < (int)eng->ops.size()) ? &eng->ops[op_id] : nullptr;
  int levels = 0;
  std::string why;
  int rc = validate(*prob, op, &levels, &why);
  if (rc != PLSQR_OK) return set_error(rc, why);
  if (prob->precision != PLSQR_PREC_FP32)
    return set_error(PLSQR_E_INVALID, "single requests run in PLSQR_PREC_FP32");
  auto r = std::make_unique<Request>();
  r->ticket = eng->next_ticket++;
  r->op_id = op_id;
  r->pb = *prob;
  r->g = g_dev;
  r->f_out = f_dev;
  r->lay = make_layout(*prob, op->op.n_y, levels, op->op.kind);
  if (eng->budget && r->lay.total > eng->budget)
    return set_error(PLSQR_E_BUDGET, "request workspace exceeds the engine's HBM budget");
  r->t_submit = now_ms();
  const uint64_t t = r->ticket;
  eng->reqs.emplace(t, std::move(r));
  // FIFO admission: the request starts now if it and everything queued before it fit
  // the budget; otherwise it waits for earlier requests to complete.
  eng->queued.push_back(t);
  progress(eng);
  *ticket = t;
  return PLSQR_OK;
}

int plsqr_poll(plsqr_engine *eng, uint64_t ticket, plsqr_result *out) {
  if (!eng) return set_error(PLSQR_E_INVALID, "null engine");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  auto it = eng->reqs.find(ticket);
  if (it == eng->reqs.end()) return set_error(PLSQR_E_UNKNOWN_TICKET, "unknown or retired ticket");
  progress(eng);
  Request &r = *it->second;
  if (r.state != Request::DONE) return PLSQR_PENDING;
  if (out) *out = r.result;
  const int st = r.status;
  eng->reqs.erase(it);
  if (st != PLSQR_OK) {
    const char *m = st == PLSQR_E_NOT_SPD ? "preconditioner not positive definite"
                    : st == PLSQR_E_NONFINITE ? "non-finite value in the Krylov scalars"
                                              : "request failed";
    set_error(st, m);
  }
  return st;
}

int plsqr_wait_all(plsqr_engine *eng) {
  if (!eng) return set_error(PLSQR_E_INVALID, "null engine");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  for (;;) {
    HIP_TRY(hipStreamSynchronize(eng->stream));
    progress(eng);
    bool running = false;
    for (auto &kv : eng->reqs) running = running || kv.second->state == Request::RUNNING;
    if (eng->queued.empty() && !running) break;
  }
  return PLSQR_OK;
}

int plsqr_destroy(plsqr_engine *eng) {
  if (!eng) return PLSQR_OK;
  {
    std::lock_guard<std::mutex> lk(eng->mu);
    DeviceGuard dg(eng->device);
    hipStreamSynchronize(eng->stream);
    eng->queued.clear();
    for (auto &kv : eng->reqs) {
      Request &r = *kv.second;
      if (r.state == Request::RUNNING) reap(eng, r);
    }
    eng->reqs.clear();
    eng->pool.trim();
  }
  delete eng;
  return PLSQR_OK;
}

const char *plsqr_last_error(const plsqr_engine *eng) {
  (void)eng;
  return g_last_error.c_str();
}

}  // extern "C"
