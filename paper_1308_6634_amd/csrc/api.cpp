// C ABI of the library (declared in include/plsqr.h): engine lifetime, operator
// registration, request submission/completion, HBM-budget admission.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <chrono>
#include <thread>
#include <tuple>

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
    for (size_t i = 0; i < op.taps.size() && i < (size_t)kMaxTaps; ++i) {
      D.taps[i] = op.taps[i];
      D.taps_rev[i] = op.taps[op.taps.size() - 1 - i];
    }
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
  D.gemv_rows = pb.tune_gemv_rows ? pb.tune_gemv_rows : 4;
  D.blur_window = pb.tune_blur_window;
  D.blur_xgroups = pb.tune_blur_xgroups;
  D.vcycle_mode = pb.tune_vcycle;
  D.zm_ty = pb.tune_zm_ty;
  D.zm_zc = pb.tune_zm_zc;
  D.zm_v = pb.tune_zm_v;
  D.tail_cells = pb.tune_tail_cells;
  D.update_site = pb.tune_update_site;
  D.out_f = r.f_out;
  D.sc = reinterpret_cast<double *>(ws + Ly.sc);
  D.part = reinterpret_cast<double *>(ws + Ly.part);
  D.cfac = reinterpret_cast<double *>(ws + Ly.cfac);
  D.diag = reinterpret_cast<double *>(ws + Ly.diag);
  D.nc = Ly.nc;
  D.stop_flags = (int)(pb.flags & (PLSQR_FLAG_STOP_S4 | PLSQR_FLAG_STOP_OUTER));
  D.s4_level = (pb.flags & PLSQR_FLAG_STOP_S4) ? pb.eta * pb.delta : 0.0;
  D.outer_rtol = pb.outer_rtol;
  D.outer_min = pb.outer_min;
  D.aw = Ly.aw ? F(Ly.aw) : nullptr;
  D.af = Ly.af ? F(Ly.af) : nullptr;
  D.outer_count = pb.outer;
  D.inner_count = pb.inner;
  if (!r.taus.empty()) {
    D.n_tau = (int)r.taus.size();
    for (int t = 0; t < D.n_tau; ++t) D.taus[t] = r.taus[t];
    D.basis = F(Ly.basis);
    D.hist = reinterpret_cast<double *>(ws + Ly.hist);
    D.tau_scr = reinterpret_cast<double *>(ws + Ly.tau_scr);
    D.ycoef = F(Ly.ycoef);
    D.f_taus = r.f_taus;
  }
  if (op.op.kind == PLSQR_OP_RING) {
    D.ring = op.ring;
    D.ringpart = F(Ly.ringpart);
    D.n_src = op.op.n_src;
    D.n_det = op.op.n_det;
    D.ring_chunk = Ly.ring_chunk;
    D.ring_chunks = Ly.ring_chunks;
    D.ring_groups = Ly.ring_groups;
    D.ringpart2 = F(Ly.ringpart2);
    D.ring_mu = (float)op.op.mu;
  }
  double eps_l = pb.eps;
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
    // Galerkin: P^T (eps I) P = (children per coarse cell) eps I, 8 while the finer level has
    // more than one z-plane, else 4
    if (l > 0) eps_l *= (Ly.lnz[l - 1] > 1) ? 8.0 : 4.0;
    L.eps = eps_l;
  }
  plan_vcycle(D, Ly);
  (void)eng;
}

// Pinned staging layout of a request: [InstDesc][scalars][per-outer records].
size_t pin_sc_off() { return (sizeof(InstDesc) + 255) / 256 * 256; }
size_t pin_dg_off() { return pin_sc_off() + SC_COUNT * sizeof(double); }
size_t pin_bytes(const plsqr_problem &pb) {
  return pin_dg_off() + (size_t)(pb.outer + 1) * DG_COUNT * sizeof(double);
}

// Group workspace: descriptor pointer array, then (MFMA path) packed operands and partials.
size_t plan_group(Group &G, const Operator &op, const Layout &Ly) {
  size_t off = 0;
  auto take = [&](size_t b) {
    off = (off + 255) / 256 * 256;
    const size_t o = off;
    off += std::max<size_t>(b, 4);
    return o;
  };
  const int B = (int)G.members.size();
  take((size_t)B * sizeof(void *));
  G.use_gemm = (G.precision != PLSQR_PREC_FP32) && op.op.kind == PLSQR_OP_DENSE;
  if (G.use_gemm) {
    GemmArgs &g = G.gemm;
    g.Bpad = B <= 32 ? 32 : 64;
    const long long m = Ly.m, n = Ly.n;
    const long long rowtiles = m / 256;      // forward GEMM blocks own 256 rows of A
    // Split K until about 256 blocks (one per compute unit) share the forward product: more
    // splits only add partial sums to write and reduce (8 splits of the 8192 x 262144 batch
    // product take 1.42 ms with its reduction, 16 take 1.45 ms, 32 take 1.54 ms). K chunks are
    // multiples of 256 (four 64-K steps of the GEMM pipeline); n % 256 == 0, so the last
    // chunk is one too.
    long long ks = std::max(1LL, std::min(n / 256, (256 + rowtiles - 1) / rowtiles));
    long long kchunk = ((n + ks - 1) / ks + 255) / 256 * 256;
    ks = (n + kchunk - 1) / kchunk;
    g.ks = (int)ks;
    g.kchunk = kchunk;
    g.use_A_lo = (G.precision == PLSQR_PREC_BF16_REFINED) ? 1 : 0;
    // offsets now, pointers after allocation
    g.X_hi = reinterpret_cast<void *>(take((size_t)g.Bpad * n * 2));
    g.X_lo = reinterpret_cast<void *>(take((size_t)g.Bpad * n * 2));
    g.U_hi = reinterpret_cast<void *>(take((size_t)g.Bpad * m * 2));
    g.U_lo = reinterpret_cast<void *>(take((size_t)g.Bpad * m * 2));
    g.Ypart = reinterpret_cast<float *>(take((size_t)g.ks * m * g.Bpad * 4));
  }
  return (off + 255) / 256 * 256;
}

// Build (once) the tiled BF16 left operands of the batched products, A (forward) and A^T
// (adjoint), each as interleaved hi/lo tile pairs owned by the library. The hi parts come from
// the caller's A_hi_dev when given, else hi = bf16(A); the lo parts from A_lo_dev when given,
// else lo = bf16(A - bf16(A)). Both parts are built whatever the precision, so one copy serves
// BF16 and BF16_REFINED groups alike.
int ensure_bf16(plsqr_engine *eng, Operator &op) {
  if (op.A_t && op.At_t) return PLSQR_OK;
  const long long m = op.op.n_y, n = (long long)op.op.nx * op.op.ny * op.op.nz;
  const size_t bytes = (size_t)m * n * 2 * 2;
  // both copies or neither: a failed allocation leaves none behind, so a later call builds
  // the pair again
  if (hipMalloc(&op.A_t, bytes) != hipSuccess || hipMalloc(&op.At_t, bytes) != hipSuccess) {
    if (op.A_t) hipFree(op.A_t);
    if (op.At_t) hipFree(op.At_t);
    op.A_t = op.At_t = nullptr;
    return set_error(PLSQR_E_NOMEM, "allocation of the BF16 operator copies failed");
  }
  const uint16_t *hi = op.op.A_hi_dev, *lo = op.op.A_lo_dev;
  for (int tr = 0; tr < 2; ++tr) {
    void *dst = tr ? op.At_t : op.A_t;
    if (!hi || !lo) launch_split_tiled(eng->stream, op.op.A_dev, m, n, tr, dst);
    if (hi) launch_retile16(eng->stream, hi, m, n, tr, 0, dst);
    if (lo) launch_retile16(eng->stream, lo, m, n, tr, 1, dst);
  }
  HIP_TRY(hipGetLastError());
  return PLSQR_OK;
}

void release_group(plsqr_engine *eng, Group &G) {
  if (G.ev_start) hipEventDestroy(G.ev_start);
  if (G.ev_end) hipEventDestroy(G.ev_end);
  G.ev_start = G.ev_end = nullptr;
  for (auto *lst : {&G.fwd_events, &G.adj_events, &G.setup_events, &G.vcycle_events,
                    &G.update_events, &G.diag_events}) {
    for (auto &e : *lst) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
    lst->clear();
  }
  for (uint64_t t : G.members) {
    auto it = eng->reqs.find(t);
    if (it == eng->reqs.end()) continue;
    Request &r = *it->second;
    if (r.ws) eng->pool.put(r.ws, r.lay.total);
    r.ws = nullptr;
    if (r.pinned) hipHostFree(r.pinned);
    r.pinned = nullptr;
  }
  if (G.gws) eng->pool.put(G.gws, G.gws_bytes);
  G.gws = nullptr;
  G.graphs.reset();
  if (G.pinned) hipHostFree(G.pinned);
  G.pinned = nullptr;
  if (G.state == Group::RUNNING) eng->used -= G.bytes;
}

// Allocate and enqueue a group (QUEUED -> RUNNING). Caller holds the lock. Nothing waits
// for earlier work on the stream: descriptors go up and results come down through
// pinned host memory with stream-ordered copies.
int start_group_impl(plsqr_engine *eng, Group &G) {
  Operator &op = eng->ops[G.op_id];
  const int B = (int)G.members.size();
  Request &r0 = *eng->reqs[G.members[0]];
  if (G.use_gemm) {
    const int rc = ensure_bf16(eng, op);
    if (rc != PLSQR_OK) return rc;
  }
  G.state = Group::RUNNING;        // from here on release_group returns the budget
  eng->used += G.bytes;
  G.gws = static_cast<char *>(eng->pool.get(G.gws_bytes));
  if (!G.gws) return set_error(PLSQR_E_NOMEM, "device allocation of the batch workspace failed");
  G.d_descs = reinterpret_cast<InstDesc **>(G.gws);
  if (G.use_gemm) {
    GemmArgs &g = G.gemm;
    auto fix = [&](void *&p) { p = G.gws + reinterpret_cast<size_t>(p); };
    fix(g.X_hi);
    fix(g.X_lo);
    fix(g.U_hi);
    fix(g.U_lo);
    g.Ypart = reinterpret_cast<float *>(G.gws + reinterpret_cast<size_t>(g.Ypart));
    g.A_t = op.A_t;
    g.At_t = op.At_t;
  }
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&G.pinned), (size_t)B * sizeof(void *),
                        hipHostMallocDefault));
  for (int b = 0; b < B; ++b) {
    Request &r = *eng->reqs[G.members[b]];
    r.ws = static_cast<char *>(eng->pool.get(r.lay.total));
    if (!r.ws) return set_error(PLSQR_E_NOMEM, "device allocation of a request workspace failed");
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&r.pinned), pin_bytes(r.pb), hipHostMallocDefault));
    fill_desc(eng, r, op);
    r.d_desc = reinterpret_cast<InstDesc *>(r.ws + r.lay.desc);
    std::memcpy(r.pinned, &r.host, sizeof(InstDesc));
    reinterpret_cast<InstDesc **>(G.pinned)[b] = r.d_desc;
  }
  HIP_TRY(hipEventCreate(&G.ev_start));
  HIP_TRY(hipEventCreate(&G.ev_end));
  HIP_TRY(hipEventRecord(G.ev_start, eng->stream));
  for (int b = 0; b < B; ++b) {
    Request &r = *eng->reqs[G.members[b]];
    HIP_TRY(hipMemcpyAsync(r.d_desc, r.pinned, sizeof(InstDesc), hipMemcpyHostToDevice, eng->stream));
  }
  HIP_TRY(hipMemcpyAsync(G.d_descs, G.pinned, (size_t)B * sizeof(void *), hipMemcpyHostToDevice,
                         eng->stream));
  BatchView bv{G.d_descs, B, &r0.host, &r0.lay, G.timed ? &G.fwd_events : nullptr,
               G.timed ? &G.adj_events : nullptr, G.use_gemm ? &G.gemm : nullptr};
  if (G.phases) {
    bv.setup_events = &G.setup_events;
    bv.vcycle_events = &G.vcycle_events;
    bv.update_events = &G.update_events;
    bv.diag_events = &G.diag_events;
  }
  if (!(r0.pb.flags & PLSQR_FLAG_NO_GRAPHS)) G.graphs = std::make_unique<GraphCache>();
  enqueue_whole_solve(eng->stream, bv, r0.pb.outer, r0.pb.inner, G.graphs.get());
  HIP_TRY(hipGetLastError());
  for (int b = 0; b < B; ++b) {
    Request &r = *eng->reqs[G.members[b]];
    HIP_TRY(hipMemcpyAsync(r.pinned + pin_sc_off(), r.ws + r.lay.sc, SC_COUNT * sizeof(double),
                           hipMemcpyDeviceToHost, eng->stream));
    HIP_TRY(hipMemcpyAsync(r.pinned + pin_dg_off(), r.ws + r.lay.diag,
                           (size_t)(r.pb.outer + 1) * DG_COUNT * sizeof(double),
                           hipMemcpyDeviceToHost, eng->stream));
  }
  HIP_TRY(hipEventRecord(G.ev_end, eng->stream));
  return PLSQR_OK;
}

void fail_group(plsqr_engine *eng, Group &G, int rc) {
  for (uint64_t t : G.members) {
    auto it = eng->reqs.find(t);
    if (it == eng->reqs.end()) continue;
    Request &r = *it->second;
    std::memset(&r.result, 0, sizeof(r.result));
    r.result.status = rc;
    r.status = rc;
    r.err = g_last_error;
    r.done = true;
  }
  G.state = Group::DONE;
}

int start_group(plsqr_engine *eng, Group &G) {
  const int rc = start_group_impl(eng, G);
  if (rc != PLSQR_OK) {
    hipStreamSynchronize(eng->stream);
    release_group(eng, G);
    fail_group(eng, G, rc);
  }
  return rc;
}

double total_ms(const EventList &lst) {
  double s = 0.0;
  for (auto &e : lst) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) s += t;
  }
  return s;
}

// Status, counts and per-outer records of a finished request from its scalar block and
// diagnostics (copied back to pinned memory at the end of the request).
void fill_records(const Request &r, const double *sc, const double *dg, plsqr_result &res) {
  res.status = (int)sc[SC_STATUS];
  // SC_OUTER counts the outer steps run (it stops advancing once the outer stop fired)
  res.outer_done = std::max(0, std::min(r.pb.outer, (int)sc[SC_OUTER]));
  res.levels = r.lay.levels;
  res.mixed_steps = r.mixed_steps;
  for (int k = 1; k <= res.outer_done; ++k) {
    res.resid[k - 1] = dg[(size_t)k * DG_COUNT + DG_RESID];
    res.penalty[k - 1] = dg[(size_t)k * DG_COUNT + DG_PENALTY];
    res.inner_done[k - 1] = (int)dg[(size_t)k * DG_COUNT + DG_INNER];
  }
}

// Collect a finished group: read every member's diagnostics, release memory.
void reap(plsqr_engine *eng, Group &G) {
  float ms = 0.f;
  if (G.ev_start && G.ev_end) hipEventElapsedTime(&ms, G.ev_start, G.ev_end);
  const double fwd = total_ms(G.fwd_events), adj = total_ms(G.adj_events);
  const double now = now_ms();
  for (uint64_t t : G.members) {
    Request &r = *eng->reqs[t];
    plsqr_result &res = r.result;
    std::memset(&res, 0, sizeof(res));
    const double *sc = reinterpret_cast<const double *>(r.pinned + pin_sc_off());
    const double *dg = reinterpret_cast<const double *>(r.pinned + pin_dg_off());
    fill_records(r, sc, dg, res);
    res.device_ms = ms;
    res.forward_ms = fwd;
    res.forward_launches = (int64_t)G.fwd_events.size();
    res.adjoint_ms = adj;
    res.adjoint_launches = (int64_t)G.adj_events.size();
    res.workspace_bytes = (int64_t)r.lay.total;
    if (G.phases) {
      res.setup_ms = total_ms(G.setup_events);
      res.vcycle_ms = total_ms(G.vcycle_events);
      res.update_ms = total_ms(G.update_events);
      res.diag_ms = total_ms(G.diag_events);
      res.phase_launches = (int64_t)G.vcycle_events.size();
    }
    r.t_done = now;
    res.submit_to_done_ms = r.t_done - r.t_submit;
    r.status = res.status;
    r.done = true;
  }
  release_group(eng, G);
  G.state = Group::DONE;
}

// Reap every finished running group, then start queued ones that now fit (FIFO).
void progress(plsqr_engine *eng) {
  for (auto it = eng->groups.begin(); it != eng->groups.end();) {
    Group &G = *it->second;
    if (G.state == Group::RUNNING && hipEventQuery(G.ev_end) == hipSuccess) reap(eng, G);
    if (G.state == Group::DONE) it = eng->groups.erase(it);
    else ++it;
  }
  while (!eng->queued.empty()) {
    auto it = eng->groups.find(eng->queued.front());
    if (it == eng->groups.end()) {
      eng->queued.pop_front();
      continue;
    }
    Group &G = *it->second;
    if (eng->budget && eng->used + G.bytes > eng->budget) break;
    eng->queued.pop_front();
    start_group(eng, G);
  }
}

// Validate and register a group of requests; returns PLSQR_OK and the tickets.
int submit_group(plsqr_engine *eng, int32_t op_id, int count, const plsqr_problem *probs,
                 const float *const *g_devs, float *const *f_devs, uint64_t *tickets,
                 const std::vector<double> *taus = nullptr, float *f_taus = nullptr) {
  const Operator *op = (op_id >= 0 && op_id < (int)eng->ops.size()) ? &eng->ops[op_id] : nullptr;
  std::vector<Layout> lays(count);
  for (int b = 0; b < count; ++b) {
    if (!g_devs[b] || !f_devs[b]) return set_error(PLSQR_E_INVALID, "g_dev and f_dev must be device pointers");
    int levels = 0;
    std::string why;
    const int rc = validate(probs[b], op, &levels, &why);
    if (rc != PLSQR_OK) return set_error(rc, why);
    lays[b] = make_layout(probs[b], op->op.n_y, levels, op->op.kind, taus ? (int)taus->size() : 0);
    const plsqr_problem &a = probs[0], &c = probs[b];
    if (c.outer != a.outer || c.inner != a.inner || lays[b].levels != lays[0].levels ||
        c.smoother != a.smoother || c.nu_pre != a.nu_pre || c.cheb_degree != a.cheb_degree ||
        c.precision != a.precision || c.flags != a.flags ||
        c.tune_gemv_rows != a.tune_gemv_rows || c.tune_col_chunks != a.tune_col_chunks ||
        c.tune_blur_window != a.tune_blur_window || c.tune_blur_xgroups != a.tune_blur_xgroups ||
        c.tune_vcycle != a.tune_vcycle || c.tune_zm_ty != a.tune_zm_ty ||
        c.tune_zm_zc != a.tune_zm_zc || c.tune_zm_v != a.tune_zm_v ||
        c.tune_tail_cells != a.tune_tail_cells || c.tune_update_site != a.tune_update_site)
      return set_error(PLSQR_E_INVALID,
                       "a batch must share counts, levels, smoother schedule, precision and flags");
  }
  const int prec = probs[0].precision;
  if (prec != PLSQR_PREC_FP32) {
    if (op->op.kind != PLSQR_OP_DENSE)
      return set_error(PLSQR_E_INVALID, "BF16 products need a dense operator");
    if (count > 64) return set_error(PLSQR_E_INVALID, "a BF16 batch holds at most 64 instances");
    if (lays[0].n % 256 || lays[0].m % 256)
      return set_error(PLSQR_E_INVALID, "BF16 products need n_X and n_Y divisible by 256");
  }
  auto G = std::make_unique<Group>();
  G->id = eng->next_group++;
  G->op_id = op_id;
  G->precision = prec;
  G->phases = (probs[0].flags & PLSQR_FLAG_TIME_PHASES) != 0;
  G->timed = G->phases || (probs[0].flags & PLSQR_FLAG_TIME_PRODUCTS) != 0;
  const double t = now_ms();
  for (int b = 0; b < count; ++b) {
    auto r = std::make_unique<Request>();
    r->ticket = eng->next_ticket++;
    r->group = G->id;
    r->pb = probs[b];
    r->g = g_devs[b];
    r->f_out = f_devs[b];
    r->lay = lays[b];
    if (taus) {
      r->taus = *taus;
      r->f_taus = f_taus;
    }
    r->t_submit = t;
    G->members.push_back(r->ticket);
    G->bytes += r->lay.total;
    tickets[b] = r->ticket;
    eng->reqs.emplace(r->ticket, std::move(r));
  }
  G->gws_bytes = plan_group(*G, *op, lays[0]);
  G->bytes += G->gws_bytes;
  if (eng->budget && G->bytes > eng->budget) {
    for (uint64_t tk : G->members) eng->reqs.erase(tk);
    return set_error(PLSQR_E_BUDGET, "request workspace exceeds the engine's HBM budget");
  }
  eng->queued.push_back(G->id);
  eng->groups.emplace(G->id, std::move(G));
  progress(eng);
  return PLSQR_OK;
}

// ------------------------------------------------------------------------------------
// Serving mode: a scheduler thread admits requests by HBM budget, keeps their Krylov and
// multigrid state resident, and every tick advances each resident request by one step
// of its fixed schedule. Requests of the same grid and multigrid schedule that are at the
// same step type form one subgroup, launched together as a batch (their blur taps,
// regulariser, tau, eps and scalars come from their own descriptors), so requests that
// arrive while others run join the next tick. Only this thread issues HIP calls.
// ------------------------------------------------------------------------------------
// Everything a subgroup's launches take from its first member: grid and hierarchy, smoother
// schedule, step type, stop flags (masks, S4 kernels), the tuned launch shapes, and for a
// dense or ring operator the operator itself (its row count sizes grids, column chunks and
// the ring adjoint's LDS). Blur requests of one grid share launches whatever their taps.
struct ClassKey {
  int nx, ny, nz, levels, smoother, nu, deg, kind, type, stop, op, gemv, cols, win, xg, vc, zty,
      zzc, zv, tail, usite;
  bool operator<(const ClassKey &o) const {
    return std::tie(nx, ny, nz, levels, smoother, nu, deg, kind, type, stop, op, gemv, cols, win,
                    xg, vc, zty, zzc, zv, tail, usite) <
           std::tie(o.nx, o.ny, o.nz, o.levels, o.smoother, o.nu, o.deg, o.kind, o.type, o.stop,
                    o.op, o.gemv, o.cols, o.win, o.xg, o.vc, o.zty, o.zzc, o.zv, o.tail, o.usite);
  }
};

void serve_collect(plsqr_engine *eng) {
  for (size_t i = 0; i < eng->finishing.size();) {
    Request &r = *eng->reqs[eng->finishing[i]];
    if (hipEventQuery(r.ev_done) != hipSuccess) {
      ++i;
      continue;
    }
    plsqr_result &res = r.result;
    std::memset(&res, 0, sizeof(res));
    const double *sc = reinterpret_cast<const double *>(r.pinned + pin_sc_off());
    const double *dg = reinterpret_cast<const double *>(r.pinned + pin_dg_off());
    fill_records(r, sc, dg, res);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.ev_start, r.ev_done) == hipSuccess) res.device_ms = ms;
    res.workspace_bytes = (int64_t)r.lay.total;
    r.t_done = now_ms();
    res.submit_to_done_ms = r.t_done - r.t_submit;
    hipEventDestroy(r.ev_start);
    hipEventDestroy(r.ev_done);
    r.ev_start = r.ev_done = nullptr;
    hipHostFree(r.pinned);
    r.pinned = nullptr;
    // the request's kernels ran on worker streams: its memory returns only now
    eng->pool.put(r.ws, r.lay.total);
    r.ws = nullptr;
    eng->used -= r.lay.total;
    r.status = res.status;
    r.done = true;
    eng->finishing[i] = eng->finishing.back();
    eng->finishing.pop_back();
  }
}

void serve_admit(plsqr_engine *eng) {
  while (!eng->serve_queue.empty()) {
    Request &r = *eng->reqs[eng->serve_queue.front()];
    if (eng->budget && eng->used + r.lay.total > eng->budget) break;
    eng->serve_queue.pop_front();
    int rc = PLSQR_OK;
    r.ws = static_cast<char *>(eng->pool.get(r.lay.total));
    if (!r.ws) rc = PLSQR_E_NOMEM;
    if (rc == PLSQR_OK &&
        hipHostMalloc(reinterpret_cast<void **>(&r.pinned), pin_bytes(r.pb), hipHostMallocDefault) != hipSuccess)
      rc = PLSQR_E_NOMEM;
    if (rc == PLSQR_OK && (hipEventCreate(&r.ev_start) != hipSuccess || hipEventCreate(&r.ev_done) != hipSuccess))
      rc = PLSQR_E_HIP;
    if (rc != PLSQR_OK) {
      if (r.ws) eng->pool.put(r.ws, r.lay.total);
      r.ws = nullptr;
      if (r.pinned) hipHostFree(r.pinned);
      r.pinned = nullptr;
      std::memset(&r.result, 0, sizeof(r.result));
      r.result.status = rc;
      r.status = rc;
      r.done = true;
      continue;
    }
    eng->used += r.lay.total;
    fill_desc(eng, r, eng->ops[r.group]);   // in serving mode `group` holds the operator id
    r.d_desc = reinterpret_cast<InstDesc *>(r.ws + r.lay.desc);
    std::memcpy(r.pinned, &r.host, sizeof(InstDesc));
    hipEventRecord(r.ev_start, eng->stream);
    hipMemcpyAsync(r.d_desc, r.pinned, sizeof(InstDesc), hipMemcpyHostToDevice, eng->stream);
    r.step = 0;
    r.steps_total = step_count(r.pb);
    eng->resident.push_back(r.ticket);
  }
}

// End every resident request with status rc (a tick could not be built). The device is
// drained first: earlier ticks may still run on their workspaces. Caller holds the lock.
void serve_fail_resident(plsqr_engine *eng, int rc, const std::string &msg) {
  hipStreamSynchronize(eng->stream);
  for (uint64_t t : eng->resident) {
    Request &r = *eng->reqs[t];
    if (r.ev_start) hipEventDestroy(r.ev_start);
    if (r.ev_done) hipEventDestroy(r.ev_done);
    r.ev_start = r.ev_done = nullptr;
    if (r.pinned) hipHostFree(r.pinned);
    r.pinned = nullptr;
    if (r.ws) {
      eng->pool.put(r.ws, r.lay.total);
      eng->used -= r.lay.total;
    }
    r.ws = nullptr;
    std::memset(&r.result, 0, sizeof(r.result));
    r.result.status = rc;
    r.status = rc;
    r.err = msg;
    r.done = true;
  }
  eng->resident.clear();
}

// Build and enqueue one tick. Caller holds the lock.
// What every instance of one ragged launch shares: the smoother schedule (the fused kernels'
// variant), the stop flags (epilogue masks) and the blur launch knobs (kernel variants).
struct RagKey {
  int smoother, nu, deg, stop, win, xg;
  bool operator<(const RagKey &o) const {
    return std::tie(smoother, nu, deg, stop, win, xg) <
           std::tie(o.smoother, o.nu, o.deg, o.stop, o.win, o.xg);
  }
};

void serve_tick(plsqr_engine *eng) {
  std::map<ClassKey, std::vector<Request *>> groups;
  // inner steps that can share launches across grids, by what such launches must share
  std::map<RagKey, std::vector<Request *>> rag_groups;
  auto class_key = [](const Request &r) {
    const plsqr_problem &pb = r.pb;
    // in serving mode `group` holds the operator id
    const int op_key = r.host.op_kind == PLSQR_OP_BLUR ? -1 : (int)r.group;
    return ClassKey{pb.nx, pb.ny, pb.nz, r.lay.levels, pb.smoother, pb.nu_pre, pb.cheb_degree,
                    r.host.op_kind, step_type(pb, r.step),
                    (int)(pb.flags & (PLSQR_FLAG_STOP_S4 | PLSQR_FLAG_STOP_OUTER)), op_key,
                    pb.tune_gemv_rows, pb.tune_col_chunks, pb.tune_blur_window,
                    pb.tune_blur_xgroups, pb.tune_vcycle, pb.tune_zm_ty, pb.tune_zm_zc,
                    pb.tune_zm_v, pb.tune_tail_cells, pb.tune_update_site};
  };
  for (uint64_t t : eng->resident) {
    Request &r = *eng->reqs[t];
    const plsqr_problem &pb = r.pb;
    if (step_type(pb, r.step) == ST_INNER && ragged_ok(r.host, r.lay)) {
      RagKey rk{pb.smoother, pb.nu_pre, pb.cheb_degree,
                (int)(pb.flags & (PLSQR_FLAG_STOP_S4 | PLSQR_FLAG_STOP_OUTER)),
                pb.tune_blur_window, pb.tune_blur_xgroups};
      rag_groups[rk].push_back(&r);
      continue;
    }
    groups[class_key(r)].push_back(&r);
  }
  // a ragged group of one class runs as a uniform batch; one of several classes runs in shared
  // launches, kMaxRag instances at a time
  std::vector<std::vector<Request *>> rag_chunks;
  rag_chunks.reserve(eng->resident.size());
  for (auto &kv : rag_groups) {
    std::vector<Request *> &mem = kv.second;
    bool one_class = true;
    for (Request *r : mem) one_class = one_class && !(class_key(*r) < class_key(*mem[0])) &&
                                       !(class_key(*mem[0]) < class_key(*r));
    if (one_class) {
      std::vector<Request *> &g = groups[class_key(*mem[0])];
      g.insert(g.end(), mem.begin(), mem.end());
      continue;
    }
    for (size_t i = 0; i < mem.size(); i += kMaxRag)
      rag_chunks.emplace_back(mem.begin() + i, mem.begin() + std::min(mem.size(), i + kMaxRag));
  }
  plsqr_engine::TickSlot &slot = eng->ring[eng->ring_next];
  const size_t need =
      eng->resident.size() * sizeof(void *) + (groups.size() + rag_chunks.size()) * 256;
  if (slot.cap < need) {
    // the slot's last tick has finished: at most max_inflight_ticks (< ring size) are queued
    if (slot.pinned) hipHostFree(slot.pinned);
    if (slot.dev) hipFree(slot.dev);
    slot.pinned = slot.dev = nullptr;
    slot.cap = 0;
    const size_t cap = std::max<size_t>(need * 2, 1 << 16);
    if (hipHostMalloc(reinterpret_cast<void **>(&slot.pinned), cap, hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&slot.dev), cap) != hipSuccess) {
      if (slot.pinned) hipHostFree(slot.pinned);
      slot.pinned = nullptr;
      slot.dev = nullptr;
      serve_fail_resident(eng, PLSQR_E_NOMEM, "allocation of a serving tick's pointer arrays failed");
      return;
    }
    slot.cap = cap;
  }
  size_t off = 0;
  struct PlanItem {
    size_t off;
    std::vector<Request *> *mem;
    bool ragged;
  };
  std::vector<PlanItem> plan;
  auto place = [&](std::vector<Request *> &mem, bool ragged) {
    off = (off + 255) / 256 * 256;
    InstDesc **dst = reinterpret_cast<InstDesc **>(slot.pinned + off);
    for (size_t i = 0; i < mem.size(); ++i) dst[i] = mem[i]->d_desc;
    plan.push_back(PlanItem{off, &mem, ragged});
    off += mem.size() * sizeof(void *);
  };
  for (auto &c : rag_chunks) place(c, true);
  for (auto &kv : groups) place(kv.second, false);
  hipMemcpyAsync(slot.dev, slot.pinned, off, hipMemcpyHostToDevice, eng->stream);
  hipEventRecord(eng->ev_upload, eng->stream);
  // subgroups run concurrently on the worker streams; each waits for the upload (which is
  // ordered after the previous tick and after new admissions on the engine stream)
  const int nl = (int)eng->lanes.size();
  std::vector<bool> used(nl, false);
  std::vector<Request *> finished;
  int gi = 0;
  for (auto &pl : plan) {
    const int li = gi++ % nl;
    hipStream_t ls = eng->lanes[li];
    if (!used[li]) {
      hipStreamWaitEvent(ls, eng->ev_upload, 0);
      used[li] = true;
    }
    std::vector<Request *> &mem = *pl.mem;
    Request &r0 = *mem[0];
    InstDesc *const *dd = reinterpret_cast<InstDesc *const *>(slot.dev + pl.off);
    if (pl.ragged) {
      const InstDesc *hs[kMaxRag];
      const Layout *ls_[kMaxRag];
      for (size_t i = 0; i < mem.size(); ++i) {
        hs[i] = &mem[i]->host;
        ls_[i] = &mem[i]->lay;
        ++mem[i]->mixed_steps;
      }
      enqueue_inner_ragged(ls, RagBatch{dd, (int)mem.size(), hs, ls_});
    } else {
      BatchView bv{dd, (int)mem.size(), &r0.host, &r0.lay, nullptr, nullptr, nullptr};
      switch (step_type(r0.pb, r0.step)) {
        case ST_BEGIN: enqueue_request_begin(ls, bv); break;
        case ST_OUTER_START:
          enqueue_outer_setup(ls, bv);
          enqueue_mlsqr_init(ls, bv);
          break;
        case ST_INNER: enqueue_inner(ls, bv); break;
        case ST_OUTER_END: enqueue_outer_end(ls, bv); break;
        default: enqueue_request_end(ls, bv); break;
      }
    }
    for (Request *r : mem) {
      if (++r->step == r->steps_total) {
        hipMemcpyAsync(r->pinned + pin_sc_off(), r->ws + r->lay.sc, SC_COUNT * sizeof(double),
                       hipMemcpyDeviceToHost, ls);
        hipMemcpyAsync(r->pinned + pin_dg_off(), r->ws + r->lay.diag,
                       (size_t)(r->pb.outer + 1) * DG_COUNT * sizeof(double),
                       hipMemcpyDeviceToHost, ls);
        hipEventRecord(r->ev_done, ls);
        finished.push_back(r);
      }
    }
  }
  for (int li = 0; li < nl; ++li) {
    if (!used[li]) continue;
    hipEventRecord(eng->lane_done[li], eng->lanes[li]);
    hipStreamWaitEvent(eng->stream, eng->lane_done[li], 0);
  }
  for (Request *r : finished) {
    eng->resident.erase(std::find(eng->resident.begin(), eng->resident.end(), r->ticket));
    eng->finishing.push_back(r->ticket);
  }
  hipEventRecord(slot.ev, eng->stream);
  eng->inflight.push_back(eng->ring_next);
  eng->ring_next = (eng->ring_next + 1) % (int)eng->ring.size();
  ++eng->ticks;
}

void serve_loop(plsqr_engine *eng) {
  hipSetDevice(eng->device);
  std::unique_lock<std::mutex> lk(eng->mu);
  while (!eng->stop_worker) {
    serve_collect(eng);
    serve_admit(eng);
    if (eng->resident.empty()) {
      if (eng->finishing.empty()) {
        eng->cv.wait_for(lk, std::chrono::milliseconds(2));
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
      continue;
    }
    // bound the work queued ahead of the device so that new arrivals join quickly
    while ((int)eng->inflight.size() >= eng->max_inflight_ticks) {
      const int s = eng->inflight.front();
      hipEvent_t ev = eng->ring[s].ev;
      lk.unlock();
      while (hipEventQuery(ev) == hipErrorNotReady) std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
      eng->inflight.pop_front();
      serve_collect(eng);
    }
    serve_tick(eng);
  }
  // drain
  lk.unlock();
  hipStreamSynchronize(eng->stream);
  lk.lock();
  eng->inflight.clear();
  serve_collect(eng);
}

int serve_start(plsqr_engine *eng) {
  eng->ring.resize(4);
  for (auto &s : eng->ring)
    if (hipEventCreate(&s.ev) != hipSuccess) return set_error(PLSQR_E_HIP, "hipEventCreate failed");
  if (hipEventCreateWithFlags(&eng->ev_upload, hipEventDisableTiming) != hipSuccess)
    return set_error(PLSQR_E_HIP, "hipEventCreate failed");
  constexpr int kLanes = 4;   // default-priority streams (the box exposes 4 hardware queues)
  eng->lanes.resize(kLanes, nullptr);
  eng->lane_done.resize(kLanes, nullptr);
  for (int i = 0; i < kLanes; ++i) {
    if (hipStreamCreateWithFlags(&eng->lanes[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&eng->lane_done[i], hipEventDisableTiming) != hipSuccess)
      return set_error(PLSQR_E_HIP, "worker stream creation failed");
  }
  eng->worker = std::thread(serve_loop, eng);
  return PLSQR_OK;
}

void serve_stop(plsqr_engine *eng) {
  {
    std::lock_guard<std::mutex> lk(eng->mu);
    eng->stop_worker = true;
  }
  eng->cv.notify_all();
  if (eng->worker.joinable()) eng->worker.join();
  for (hipStream_t l : eng->lanes)
    if (l) hipStreamSynchronize(l);
  for (auto &s : eng->ring) {
    if (s.ev) hipEventDestroy(s.ev);
    if (s.pinned) hipHostFree(s.pinned);
    if (s.dev) hipFree(s.dev);
  }
  eng->ring.clear();
  for (size_t i = 0; i < eng->lanes.size(); ++i) {
    if (eng->lane_done[i]) hipEventDestroy(eng->lane_done[i]);
    if (eng->lanes[i]) hipStreamDestroy(eng->lanes[i]);
  }
  eng->lanes.clear();
  eng->lane_done.clear();
  if (eng->ev_upload) hipEventDestroy(eng->ev_upload);
  eng->ev_upload = nullptr;
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
  if (op_kind != PLSQR_OP_BLUR && op_kind != PLSQR_OP_DENSE && op_kind != PLSQR_OP_RING) return 0;
  if (op_kind == PLSQR_OP_RING && n_y > kRingMaxRows) return 0;
  // the full problem validation against an operator of this kind on the problem's grid
  Operator op;
  op.op.kind = op_kind;
  op.op.nx = prob->nx;
  op.op.ny = prob->ny;
  op.op.nz = prob->nz;
  op.op.n_y = n_y;
  int levels = 0;
  std::string why;
  if (validate(*prob, &op, &levels, &why) != PLSQR_OK) return 0;
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
  {
    // the no-allocation entry point's scratch on this device: its address is looked up once
    DeviceGuard dg(device);
    std::string why;
    const int rc = resolve_scratch(device, &why);
    if (rc != PLSQR_OK) return set_error(rc, why);
  }
  auto *e = new plsqr_engine();
  e->device = device;
  e->stream = static_cast<hipStream_t>(hip_stream);
  e->budget = hbm_budget_bytes;
  e->flags = flags;
  if (flags & PLSQR_ENGINE_SERVE) {
    const int rc = serve_start(e);
    if (rc != PLSQR_OK) {
      delete e;
      return rc;
    }
  }
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
  } else if (op->kind == PLSQR_OP_RING) {
    if (op->n_src < 1 || op->n_det < 1 || (int64_t)op->n_src * op->n_det > kRingMaxRows)
      return set_error(PLSQR_E_INVALID, "ring operator needs n_src, n_det >= 1, n_src * n_det <= 16384");
    if (!op->src_xyz || !op->det_xyz) return set_error(PLSQR_E_INVALID, "ring positions are NULL");
    if (!(op->mu > 0.0 && std::isfinite(op->mu))) return set_error(PLSQR_E_INVALID, "ring mu must be > 0");
    std::vector<float> geo(op->src_xyz, op->src_xyz + 3 * op->n_src);
    geo.insert(geo.end(), op->det_xyz, op->det_xyz + 3 * op->n_det);
    for (float c : geo)
      if (!std::isfinite(c)) return set_error(PLSQR_E_INVALID, "ring positions must be finite");
    DeviceGuard dg(eng->device);
    if (hipMalloc(&o.ring, geo.size() * sizeof(float)) != hipSuccess)
      return set_error(PLSQR_E_NOMEM, "allocation of the ring positions failed");
    if (hipMemcpy(o.ring, geo.data(), geo.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(o.ring);
      return set_error(PLSQR_E_HIP, "copy of the ring positions failed");
    }
    o.op.n_y = (int64_t)op->n_src * op->n_det;
    o.op.src_xyz = o.op.det_xyz = nullptr;
    o.op.A_dev = nullptr;
    o.op.A_hi_dev = o.op.A_lo_dev = nullptr;
  } else {
    return set_error(PLSQR_E_INVALID, "unknown operator kind");
  }
  eng->ops.push_back(o);
  *op_id = (int32_t)eng->ops.size() - 1;
  return PLSQR_OK;
}

int plsqr_solve_taus(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob,
                     const float *g_dev, float *f_dev, int32_t n_tau, const double *taus,
                     float *f_taus_dev, uint64_t *ticket) {
  if (!eng || !prob || !ticket || !taus) return set_error(PLSQR_E_INVALID, "null argument");
  if (eng->flags & PLSQR_ENGINE_SERVE)
    return set_error(PLSQR_E_INVALID, "a serving engine takes single-damping requests");
  if (prob->precision != PLSQR_PREC_FP32)
    return set_error(PLSQR_E_INVALID, "single requests run in PLSQR_PREC_FP32");
  if (n_tau < 1 || n_tau > kMaxTaus) return set_error(PLSQR_E_INVALID, "n_tau must be in [1, 64]");
  if (!f_taus_dev) return set_error(PLSQR_E_INVALID, "f_taus_dev must be a device pointer");
  if (prob->inner > kMaxTauInner) return set_error(PLSQR_E_INVALID, "a multi-tau solve takes inner <= 1024");
  if (prob->flags & (PLSQR_FLAG_STOP_S4 | PLSQR_FLAG_STOP_OUTER))
    return set_error(PLSQR_E_INVALID, "a multi-tau solve runs fixed counts (no stop flags)");
  std::vector<double> tv(taus, taus + n_tau);
  for (double t : tv)
    if (!(t >= 0.0 && std::isfinite(t))) return set_error(PLSQR_E_INVALID, "every tau must be >= 0 and finite");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  return submit_group(eng, op_id, 1, prob, &g_dev, &f_dev, ticket, &tv, f_taus_dev);
}

int plsqr_solve(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob, const float *g_dev,
                float *f_dev, uint64_t *ticket) {
  if (!eng || !prob || !ticket) return set_error(PLSQR_E_INVALID, "null argument");
  if (prob->precision != PLSQR_PREC_FP32)
    return set_error(PLSQR_E_INVALID, "single requests run in PLSQR_PREC_FP32");
  std::lock_guard<std::mutex> lk(eng->mu);
  if (eng->flags & PLSQR_ENGINE_SERVE) {
    // serving: validate and queue; the scheduler thread admits and runs it
    const Operator *op = (op_id >= 0 && op_id < (int)eng->ops.size()) ? &eng->ops[op_id] : nullptr;
    if (!g_dev || !f_dev) return set_error(PLSQR_E_INVALID, "g_dev and f_dev must be device pointers");
    int levels = 0;
    std::string why;
    const int rc = validate(*prob, op, &levels, &why);
    if (rc != PLSQR_OK) return set_error(rc, why);
    auto r = std::make_unique<Request>();
    r->ticket = eng->next_ticket++;
    r->group = (uint64_t)op_id;
    r->pb = *prob;
    r->g = g_dev;
    r->f_out = f_dev;
    r->lay = make_layout(*prob, op->op.n_y, levels, op->op.kind);
    r->host.op_kind = op->op.kind;
    if (eng->budget && r->lay.total > eng->budget)
      return set_error(PLSQR_E_BUDGET, "request workspace exceeds the engine's HBM budget");
    r->t_submit = now_ms();
    *ticket = r->ticket;
    eng->serve_queue.push_back(r->ticket);
    eng->reqs.emplace(r->ticket, std::move(r));
    eng->cv.notify_all();
    return PLSQR_OK;
  }
  DeviceGuard dg(eng->device);
  return submit_group(eng, op_id, 1, prob, &g_dev, &f_dev, ticket);
}

int plsqr_solve_batch(plsqr_engine *eng, int32_t op_id, int32_t count, const plsqr_problem *probs,
                      const float *const *g_devs, float *const *f_devs, uint64_t *tickets) {
  if (!eng || !probs || !g_devs || !f_devs || !tickets) return set_error(PLSQR_E_INVALID, "null argument");
  if (count < 1) return set_error(PLSQR_E_INVALID, "count must be >= 1");
  if (eng->flags & PLSQR_ENGINE_SERVE)
    return set_error(PLSQR_E_INVALID, "a serving engine batches by itself: submit with plsqr_solve");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  return submit_group(eng, op_id, count, probs, g_devs, f_devs, tickets);
}

int plsqr_solve_static(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob,
                       const float *g_dev, float *f_dev, plsqr_result *out) {
  if (!eng || !prob) return set_error(PLSQR_E_INVALID, "null argument");
  if (!g_dev || !f_dev) return set_error(PLSQR_E_INVALID, "g_dev and f_dev must be device pointers");
  if (eng->flags & PLSQR_ENGINE_SERVE)
    return set_error(PLSQR_E_INVALID, "plsqr_solve_static runs on a plain engine, not a serving one");
  if (prob->precision != PLSQR_PREC_FP32)
    return set_error(PLSQR_E_INVALID, "plsqr_solve_static runs in PLSQR_PREC_FP32");
  if (prob->flags & (PLSQR_FLAG_TIME_PRODUCTS | PLSQR_FLAG_TIME_PHASES))
    return set_error(PLSQR_E_INVALID, "plsqr_solve_static records no timings (they need events)");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  const Operator *op = (op_id >= 0 && op_id < (int)eng->ops.size()) ? &eng->ops[op_id] : nullptr;
  int levels = 0;
  std::string why;
  const int rc = validate(*prob, op, &levels, &why);
  if (rc != PLSQR_OK) return set_error(rc, why);
  Request r;
  r.pb = *prob;
  r.g = g_dev;
  r.f_out = f_dev;
  r.lay = make_layout(*prob, op->op.n_y, levels, op->op.kind);
  if (r.lay.total > (size_t)PLSQR_STATIC_SCRATCH_BYTES)
    return set_error(PLSQR_E_BUDGET, "the request needs " + std::to_string(r.lay.total) +
                                         " bytes of workspace, more than the " +
                                         std::to_string((size_t)PLSQR_STATIC_SCRATCH_BYTES) +
                                         "-byte static scratch of plsqr_solve_static");
  r.ws = static_cast<char *>(scratch_ptr(eng->device));
  if (!r.ws) return set_error(PLSQR_E_HIP, "the static scratch of this device was not resolved");
  fill_desc(eng, r, *op);
  InstDesc *d_desc = reinterpret_cast<InstDesc *>(r.ws + r.lay.desc);
  InstDesc **d_ptrs = reinterpret_cast<InstDesc **>(r.ws + r.lay.descptr);
  const int n_rec = (prob->outer + 1) * DG_COUNT;
  launch_static_setup(eng->stream, r.host, d_desc, d_ptrs, reinterpret_cast<double *>(r.ws + r.lay.diag),
                      n_rec);
  BatchView bv{d_ptrs, 1, &r.host, &r.lay, nullptr, nullptr, nullptr};
  enqueue_whole_solve(eng->stream, bv, prob->outer, prob->inner, nullptr);
  HIP_TRY(hipGetLastError());
  if (!out) return PLSQR_OK;
  HIP_TRY(hipStreamSynchronize(eng->stream));
  double sc[SC_COUNT];
  double dg_rec[(PLSQR_MAX_OUTER + 1) * DG_COUNT];
  HIP_TRY(hipMemcpy(sc, r.ws + r.lay.sc, sizeof(sc), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(dg_rec, r.ws + r.lay.diag, (size_t)n_rec * sizeof(double), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  fill_records(r, sc, dg_rec, *out);
  out->workspace_bytes = (int64_t)r.lay.total;
  if (out->status != PLSQR_OK)
    return set_error(out->status, out->status == PLSQR_E_NOT_SPD ? "preconditioner not positive definite"
                                  : out->status == PLSQR_E_NONFINITE ? "non-finite value in the Krylov scalars"
                                                                     : "request failed");
  return PLSQR_OK;
}

int plsqr_poll(plsqr_engine *eng, uint64_t ticket, plsqr_result *out) {
  if (!eng) return set_error(PLSQR_E_INVALID, "null engine");
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  auto it = eng->reqs.find(ticket);
  if (it == eng->reqs.end()) return set_error(PLSQR_E_UNKNOWN_TICKET, "unknown or retired ticket");
  if (!(eng->flags & PLSQR_ENGINE_SERVE)) progress(eng);
  Request &r = *it->second;
  if (!r.done) return PLSQR_PENDING;
  if (out) *out = r.result;
  const int st = r.status;
  const std::string err = r.err;
  eng->reqs.erase(it);
  if (st != PLSQR_OK) {
    const std::string m = st == PLSQR_E_NOT_SPD ? "preconditioner not positive definite"
                          : st == PLSQR_E_NONFINITE ? "non-finite value in the Krylov scalars"
                          : !err.empty()            ? err
                                                    : "request failed";
    set_error(st, m);
  }
  return st;
}

int plsqr_wait_all(plsqr_engine *eng) {
  if (!eng) return set_error(PLSQR_E_INVALID, "null engine");
  if (eng->flags & PLSQR_ENGINE_SERVE) {
    for (;;) {
      {
        std::lock_guard<std::mutex> lk(eng->mu);
        if (eng->serve_queue.empty() && eng->resident.empty() && eng->finishing.empty()) break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    return PLSQR_OK;
  }
  std::lock_guard<std::mutex> lk(eng->mu);
  DeviceGuard dg(eng->device);
  for (;;) {
    HIP_TRY(hipStreamSynchronize(eng->stream));
    progress(eng);
    if (eng->queued.empty() && eng->groups.empty()) break;
  }
  return PLSQR_OK;
}

int plsqr_destroy(plsqr_engine *eng) {
  if (!eng) return PLSQR_OK;
  if (eng->flags & PLSQR_ENGINE_SERVE) {
    serve_stop(eng);
    std::lock_guard<std::mutex> lk(eng->mu);
    for (uint64_t t : eng->resident) {
      Request &r = *eng->reqs[t];
      if (r.ws) eng->pool.put(r.ws, r.lay.total);
      r.ws = nullptr;
    }
    for (auto &kv : eng->reqs) {
      Request &r = *kv.second;
      if (r.pinned) hipHostFree(r.pinned);
      if (r.ev_start) hipEventDestroy(r.ev_start);
      if (r.ev_done) hipEventDestroy(r.ev_done);
      r.pinned = nullptr;
    }
  }
  {
    std::lock_guard<std::mutex> lk(eng->mu);
    DeviceGuard dg(eng->device);
    hipStreamSynchronize(eng->stream);
    eng->queued.clear();
    for (auto &kv : eng->groups) {
      Group &G = *kv.second;
      if (G.state == Group::RUNNING) reap(eng, G);
    }
    eng->groups.clear();
    eng->reqs.clear();
    for (auto &op : eng->ops) {
      if (op.A_t) hipFree(op.A_t);
      if (op.At_t) hipFree(op.At_t);
      if (op.ring) hipFree(op.ring);
    }
    eng->ops.clear();
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
