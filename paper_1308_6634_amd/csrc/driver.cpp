// Solve driver: the kernel sequence of Algorithm 3 around Algorithm 2, for one instance
// or for a lockstep batch of same-shaped instances. No host/device synchronisation
// happens inside: every scalar of the Krylov recurrence lives in device memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "engine.hpp"

namespace plsqr {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int validate(const plsqr_problem &pb, const Operator *op, int *levels_out, std::string *why) {
  auto bad = [&](const char *m) {
    *why = m;
    return PLSQR_E_INVALID;
  };
  if (!op) return bad("unknown operator id");
  if (pb.nx < 1 || pb.ny < 1 || pb.nz < 1) return bad("grid extents must be >= 1");
  if ((long long)pb.nx * pb.ny * pb.nz >= (1LL << 31)) return bad("grids hold fewer than 2^31 cells");
  if (pb.nx != op->op.nx || pb.ny != op->op.ny || pb.nz != op->op.nz)
    return bad("problem grid differs from the operator's grid");
  if (pb.reg < PLSQR_REG_TIKHONOV || pb.reg > PLSQR_REG_PM_EXP) return bad("unknown regulariser");
  if (pb.reg != PLSQR_REG_TIKHONOV && !(pb.T > 0.0 && std::isfinite(pb.T)))
    return bad("T must be positive and finite");
  if (!(pb.tau >= 0.0 && std::isfinite(pb.tau))) return bad("tau must be >= 0 and finite");
  if (!(pb.eps > 0.0 && std::isfinite(pb.eps))) return bad("eps must be positive and finite");
  if (pb.outer < 1 || pb.outer > PLSQR_MAX_OUTER) return bad("outer must be in [1, 64]");
  if (pb.inner < 1 || pb.inner > 1000000) return bad("inner must be in [1, 1e6]");
  if (pb.nu_pre < 1 || pb.nu_pre != pb.nu_post)
    return bad("nu_pre must equal nu_post and be >= 1 (symmetric V-cycle)");
  if (pb.smoother == PLSQR_SMOOTH_JACOBI) {
    if (!(pb.omega > 0.0 && pb.omega <= 1.0)) return bad("Jacobi omega must be in (0, 1]");
  } else if (pb.smoother == PLSQR_SMOOTH_CHEBYSHEV) {
    if (pb.cheb_degree < 1 || pb.cheb_degree > kMaxChebDegree)
      return bad("cheb_degree must be in [1, 16]");
    if (!(pb.cheb_lo > 0.0 && pb.cheb_hi > pb.cheb_lo && pb.cheb_hi <= 4.0))
      return bad("Chebyshev interval must satisfy 0 < lo < hi <= 4");
  } else {
    return bad("unknown smoother");
  }
  if (pb.precision != PLSQR_PREC_FP32 && pb.precision != PLSQR_PREC_BF16_REFINED &&
      pb.precision != PLSQR_PREC_BF16)
    return bad("unknown precision");
  if (pb.tune_gemv_rows && pb.tune_gemv_rows != 1 && pb.tune_gemv_rows != 2 &&
      pb.tune_gemv_rows != 4 && pb.tune_gemv_rows != 8)
    return bad("tune_gemv_rows must be 0, 1, 2, 4 or 8");
  if (pb.tune_col_chunks < 0 || pb.tune_col_chunks > 64) return bad("tune_col_chunks must be in [0, 64]");
  if (pb.tune_blur_window && pb.tune_blur_window != 4 && pb.tune_blur_window != 8 &&
      pb.tune_blur_window != 16 && pb.tune_blur_window != 32)
    return bad("tune_blur_window must be 0, 4, 8, 16 or 32");
  if (pb.tune_blur_xgroups && pb.tune_blur_xgroups != 1 && pb.tune_blur_xgroups != 2 &&
      pb.tune_blur_xgroups != 4)
    return bad("tune_blur_xgroups must be 0, 1, 2 or 4");
  if (pb.tune_vcycle != PLSQR_VCYCLE_FUSED && pb.tune_vcycle != PLSQR_VCYCLE_PER_SWEEP)
    return bad("tune_vcycle must be PLSQR_VCYCLE_FUSED or PLSQR_VCYCLE_PER_SWEEP");
  if (pb.tune_zm_ty && (pb.tune_zm_ty < 2 || pb.tune_zm_ty > 64 || (pb.tune_zm_ty & 1)))
    return bad("tune_zm_ty must be 0 or even in [2, 64]");
  if (pb.tune_zm_zc && (pb.tune_zm_zc < 2 || pb.tune_zm_zc > 64 || (pb.tune_zm_zc & 1)))
    return bad("tune_zm_zc must be 0 or even in [2, 64]");
  if (pb.tune_zm_v != 0 && pb.tune_zm_v != 1 && pb.tune_zm_v != 4)
    return bad("tune_zm_v must be 0, 1 or 4");
  if (pb.tune_tail_cells < 0 || pb.tune_tail_cells > (1 << 20))
    return bad("tune_tail_cells must be in [0, 2^20]");
  if (pb.tune_update_site != PLSQR_UPDATE_AUTO && pb.tune_update_site != PLSQR_UPDATE_PRODUCT &&
      pb.tune_update_site != PLSQR_UPDATE_TAIL)
    return bad("tune_update_site must be PLSQR_UPDATE_AUTO, _PRODUCT or _TAIL");
  int levels = pb.mg_levels;
  if (levels == 0) levels = plsqr_auto_levels(pb.nx, pb.ny, pb.nz);
  if (levels < 1 || levels > kMaxLevels) return bad("mg_levels out of range");
  long long nx = pb.nx, ny = pb.ny, nz = pb.nz;
  for (int l = 1; l < levels; ++l) {
    if ((nx & 1) || (ny & 1) || (nz > 1 && (nz & 1)))
      return bad("each coarsening needs even nx, ny (and nz in 3D)");
    nx /= 2;
    ny /= 2;
    if (nz > 1) nz /= 2;
  }
  if (nx * ny * nz > PLSQR_MAX_COARSE) return bad("coarsest grid has more than 512 cells");
  if (op->op.kind == PLSQR_OP_BLUR && 2 * op->op.radius + 1 > kMaxTaps) return bad("radius too large");
  if (pb.flags & PLSQR_FLAG_STOP_S4) {
    if (!(pb.eta > 0.0 && std::isfinite(pb.eta))) return bad("S4 needs eta > 0");
    if (!(pb.delta >= 0.0 && std::isfinite(pb.delta))) return bad("S4 needs a finite delta >= 0");
  }
  if (pb.flags & PLSQR_FLAG_STOP_OUTER) {
    if (!std::isfinite(pb.outer_rtol) || pb.outer_rtol < -1.0 || pb.outer_rtol >= 1.0)
      return bad("outer_rtol must be in [-1, 1)");
    if (pb.outer_min < 2) return bad("the outer stop compares R(f^k) with R(f^{k-1}): outer_min >= 2");
  }
  *levels_out = levels;
  return PLSQR_OK;
}

Layout make_layout(const plsqr_problem &pb, long long n_y, int levels, int op_kind, int n_tau) {
  Layout L;
  L.levels = levels;
  L.n = (long long)pb.nx * pb.ny * pb.nz;
  L.m = n_y;
  const bool dense = (op_kind == PLSQR_OP_DENSE);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += std::max<size_t>(bytes, 4);
    return o;
  };
  L.lnx[0] = pb.nx;
  L.lny[0] = pb.ny;
  L.lnz[0] = pb.nz;
  for (int l = 0; l < levels; ++l) {
    if (l > 0) {
      L.lnx[l] = L.lnx[l - 1] / 2;
      L.lny[l] = L.lny[l - 1] / 2;
      L.lnz[l] = L.lnz[l - 1] > 1 ? L.lnz[l - 1] / 2 : 1;
    }
    L.ln[l] = (long long)L.lnx[l] * L.lny[l] * L.lnz[l];
  }
  L.nc = (int)L.ln[levels - 1];
  const long long nb = (L.n + kBlock - 1) / kBlock;
  const long long mb = (L.m + kBlock - 1) / kBlock;
  const long long mr = (L.m + 3) / 4;
  // the strip-tiled blur passes write one partial per tile (64 x-columns x 64 along y or z)
  const long long txn = (pb.nx + 63) / 64;           // strip tiles: 64 x-columns x >= 16 deep
  const long long ty_tiles = txn * ((pb.ny + 15) / 16) * pb.nz;
  const long long tz_tiles = txn * ((pb.nz + 15) / 16) * pb.ny;
  const long long mr1 = L.m;                          // one row per block at the finest tiling
  L.nparts = (int)std::max({nb, mb, mr, mr1, ty_tiles, tz_tiles, 1LL});
  L.desc = take(sizeof(InstDesc));
  L.descptr = take(sizeof(void *));
  L.sc = take(SC_COUNT * sizeof(double));
  L.diag = take((size_t)(pb.outer + 1) * DG_COUNT * sizeof(double));
  L.part = take((size_t)L.nparts * sizeof(double));
  L.cfac = take((size_t)3 * L.nc * L.nc * sizeof(double));   // factor, L^{-1}, A^{-1}
  const size_t vb = (size_t)L.n * sizeof(float);
  L.f = take(vb);
  L.p = take(vb);
  L.v = take(vb);
  L.w = take(vb);
  L.kappa = take(vb);
  L.u = take((size_t)L.m * sizeof(float));
  if (pb.flags & PLSQR_FLAG_STOP_S4) {
    L.aw = take((size_t)L.m * sizeof(float));
    L.af = take((size_t)L.m * sizeof(float));
  }
  if (n_tau > 0) {
    L.basis = take((size_t)pb.inner * L.n * sizeof(float));
    L.hist = take((size_t)2 * (pb.inner + 1) * sizeof(double));
    L.tau_scr = take((size_t)n_tau * pb.inner * 3 * sizeof(double));
    L.ycoef = take((size_t)n_tau * pb.inner * sizeof(float));
  }
  L.colchunks = 0;
  if (op_kind == PLSQR_OP_RING) {
    // forward product: one block per chunk of voxels (a multiple of the 32-voxel staging step)
    // writes all n_Y partial sums; about 1024 blocks per instance keep 4 waves per SIMD
    long long ch = (L.n + 1023) / 1024;
    ch = std::max(32LL, (ch + 31) / 32 * 32);
    L.ring_chunk = (int)ch;
    L.ring_chunks = (int)((L.n + ch - 1) / ch);
    L.ringpart = take((size_t)L.ring_chunks * L.m * sizeof(float));
    L.ring_groups = std::min(L.ring_chunks, 32);
    L.ringpart2 = take((size_t)L.ring_groups * L.m * sizeof(float));
  } else if (!dense) {
    L.tmp1 = take(vb);
    L.tmp2 = take(vb);
  } else {
    // dense adjoint row chunks: aim for >= 2048 blocks in total
    const long long colblocks = (L.n + 4 * kBlock - 1) / (4 * kBlock);
    long long ch = pb.tune_col_chunks ? pb.tune_col_chunks : (2048 + colblocks - 1) / colblocks;
    ch = std::max(1LL, std::min({ch, 64LL, L.m}));
    L.colchunks = (int)ch;
    L.colpart = take((size_t)ch * vb);
  }
  for (int l = 0; l < levels; ++l) {
    const size_t b = (size_t)L.ln[l] * sizeof(float);
    if (l > 0) {
      L.lvl[l][0] = take(b);  // x
      L.lvl[l][1] = take(b);  // b
    }
    L.lvl[l][2] = take(b);    // r
    L.lvl[l][3] = take(b);    // t
    L.lvl[l][4] = take(b);    // s
    if (l > 0) {
      L.lvl[l][5] = take(b);  // wx
      L.lvl[l][6] = take(b);  // wy
      if (L.lnz[l] > 1) L.lvl[l][7] = take(b);  // wz
    }
    L.lvl[l][8] = take(b);    // dinv
  }
  L.total = align_up(off, 256);
  return L;
}

// ---------------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------------
static void time_begin(hipStream_t st, EventList *ev, hipEvent_t *a) {
  if (!ev) return;
  hipEventCreate(a);
  hipEventRecord(*a, st);
}
static void time_end(hipStream_t st, EventList *ev, hipEvent_t a) {
  if (!ev) return;
  hipEvent_t b;
  hipEventCreate(&b);
  hipEventRecord(b, st);
  ev->emplace_back(a, b);
}

// upd: the product applies a pending f, w update (fused_update): its first pass, or its second
// when the first carries a finaliser block. fin >= 0 (fin_blocks): the first pass (the x pass)
// also runs finaliser fin on the fin_n partials of the launch before it, in a block of its own.
static int blur_chain(hipStream_t st, const BatchView &bv, int src, int adj, int epi, int upd = 0,
                      int fin = -1, int fin_n = 0) {
  const InstDesc &H = *bv.h;
  int axes[3], na = 0;
  const int ext[3] = {H.nx, H.ny, H.nz};
  for (int a = 0; a < 3; ++a)
    if (ext[a] > 1) axes[na++] = a;
  if (na == 0) axes[na++] = 0;
  int cur = src, np = 0;
  for (int i = 0; i < na; ++i) {
    const bool last = (i == na - 1);
    const int dst = last ? V_TMP2 : ((i % 2 == 0) ? V_TMP1 : V_TMP2);
    const int e = last ? epi : (EPI_STORE | (epi & (EPI_MASK_INNER | EPI_MASK_OUTER)));
    const int u = (i == (fin >= 0 ? 1 : 0)) ? upd : 0;
    if (axes[i] == 0)
      np = launch_blur_x(st, bv.d_descs, bv.B, H.n, H.nx, cur, dst, adj, e, H.blur_xgroups, kNoRag,
                         u, i == 0 ? fin : -1, fin_n);
    else
      np = launch_blur_axis(st, bv.d_descs, bv.B, H.nx, H.ny, H.nz, axes[i], cur, dst, adj, e,
                            H.blur_window, kNoRag, u);
    cur = dst;
  }
  return np;
}

// With adaptive stops, the mask bit that lets an instance skip a product: inner products once
// its MLSQR has ended, the per-outer residual product once its outer loop has ended.
static int with_mask(const InstDesc &H, int epi) {
  if (!H.stop_flags) return epi;
  return epi | (epi == EPI_RESID ? EPI_MASK_OUTER : EPI_MASK_INNER);
}

// Whether the f, w update of an inner step is applied by the first kernel of the next forward
// product, which reads v anyway (f and w are not touched by the product), instead of a launch of
// its own: the x pass of a blur operator with four voxels per thread or the packing of the
// batched MFMA product, with the fused V-cycle schedule and no S4 recurrence or stored basis
// (they run right after the update). The update of the last inner step runs before the
// per-outer residual, which reads f.
static bool fused_update(const BatchView &bv) {
  const InstDesc &H = *bv.h;
  if (H.n_tau > 0 || (H.stop_flags & PLSQR_FLAG_STOP_S4) || H.vcycle_mode == PLSQR_VCYCLE_PER_SWEEP)
    return false;
  // the blur x pass (four voxels per thread) or the packing of the batched MFMA product
  return (H.op_kind == PLSQR_OP_BLUR && H.nx % 4 == 0) || (H.op_kind == PLSQR_OP_DENSE && bv.gemm);
}

// y = A x from vector `src`, epilogue `epi`; returns the partial count. upd: a forward product of
// an inner step, which applies the previous step's pending update when fused_update holds.
// fin, fin_n: a finaliser block in the first pass (blur operators under fin_blocks).
static int enqueue_forward(hipStream_t st, const BatchView &bv, int src, int epi, bool upd = false,
                           int fin = -1, int fin_n = 0) {
  const InstDesc &H = *bv.h;
  hipEvent_t a = nullptr;
  EventList *ev = (epi == EPI_FWD) ? bv.prod_events : nullptr;
  time_begin(st, ev, &a);
  int np;
  const int em = with_mask(H, epi);
  if (H.op_kind == PLSQR_OP_BLUR)
    np = blur_chain(st, bv, src, 0, em, (upd && fused_update(bv)) ? 1 : 0, fin, fin_n);
  else if (H.op_kind == PLSQR_OP_RING)
    np = launch_ring_forward(st, bv.d_descs, bv.B, H, src, em);
  else if (bv.gemm)
    np = launch_gemm_forward(st, bv.d_descs, bv.B, *bv.gemm, H.m, H.n, src, em,
                             (upd && fused_update(bv)) ? 1 : 0);
  else
    np = launch_gemv_rows(st, bv.d_descs, bv.B, H.m, src, em, H.gemv_rows);
  time_end(st, ev, a);
  return np;
}

// p <- su A^T u (- beta sv p). fin, fin_n: a finaliser block in the first pass (blur operators
// under fin_blocks).
static void enqueue_adjoint(hipStream_t st, const BatchView &bv, int epi, int fin = -1,
                            int fin_n = 0) {
  const InstDesc &H = *bv.h;
  hipEvent_t a = nullptr;
  EventList *ev = (epi == EPI_ADJ) ? bv.adj_events : nullptr;
  time_begin(st, ev, &a);
  const int em = with_mask(H, epi);
  if (H.op_kind == PLSQR_OP_BLUR) {
    blur_chain(st, bv, V_U, 1, em, 0, fin, fin_n);
  } else if (H.op_kind == PLSQR_OP_RING) {
    launch_ring_adjoint(st, bv.d_descs, bv.B, H, em);
  } else if (bv.gemm) {
    launch_gemm_adjoint(st, bv.d_descs, bv.B, *bv.gemm, H.m, H.n, em);
  } else {
    launch_gemv_cols(st, bv.d_descs, bv.B, H.n, H.colchunks);
    launch_colsum(st, bv.d_descs, bv.B, H.n, em);
  }
  time_end(st, ev, a);
}

// ---------------------------------------------------------------------------------
// V-cycle: v = B p; returns the partial count of the alpha^2 = v.p reduction
// ---------------------------------------------------------------------------------
static int other(int s) { return s == LB_X ? LB_T : LB_X; }
static int other_d(int s) { return s == LB_T ? LB_S : LB_T; }

// Level kernels: the four-voxel-per-thread forms where the level's rows split into 16-byte
// groups (nx % 4 == 0), the one-voxel forms otherwise; both compute the same values.
namespace {
struct LevelLaunch {
  hipStream_t st;
  InstDesc *const *d;
  int B;
  const Layout &Ly;
  bool v4(int l) const { return Ly.lnx[l] % 4 == 0; }
  long long n(int l) const { return Ly.ln[l]; }
  int jacobi(int l, int first, int src, int dst, int want) const {
    return v4(l) ? launch_jacobi4(st, d, B, l, n(l), first, src, dst, want)
                 : launch_jacobi(st, d, B, l, n(l), first, src, dst, want);
  }
  int jacobi_first2(int l, int dst, int want) const {
    return v4(l) ? launch_jacobi_first2_4(st, d, B, l, n(l), dst, want)
                 : launch_jacobi_first2(st, d, B, l, n(l), dst, want);
  }
  int jacobi_prolong(int l, int src, int dst, int want) const {
    return v4(l) ? launch_jacobi_prolong4(st, d, B, l, n(l), src, dst, want)
                 : launch_jacobi_prolong(st, d, B, l, n(l), src, dst, want);
  }
  void cheb_first(int l, int last, int dn) const {
    if (v4(l)) launch_cheb_first4(st, d, B, l, n(l), last, dn);
    else launch_cheb_first(st, d, B, l, n(l), last, dn);
  }
  void cheb_start(int l, int zero_x, int dsel) const {
    if (v4(l)) launch_cheb_start4(st, d, B, l, n(l), zero_x, dsel);
    else launch_cheb_start(st, d, B, l, n(l), zero_x, dsel);
  }
  void cheb_start_prolong(int l, int dsel) const {
    if (v4(l)) launch_cheb_start_prolong4(st, d, B, l, n(l), dsel);
    else launch_cheb_start_prolong(st, d, B, l, n(l), dsel);
  }
  int cheb_step(int l, int set_x, int upd, int last, int dsel, int dn, int step, int want,
                int add_prolong) const {
    return v4(l) ? launch_cheb_step4(st, d, B, l, n(l), set_x, upd, last, dsel, dn, step, want,
                                     add_prolong)
                 : launch_cheb_step(st, d, B, l, n(l), set_x, upd, last, dsel, dn, step, want,
                                    add_prolong);
  }
  void restrict_to(int l, int x_sel, int use_r) const {
    const int nchild = (Ly.lnz[0] > 1) ? 8 : 4;
    if (v4(l)) launch_restrict4(st, d, B, l, n(l + 1), x_sel, use_r);
    else launch_restrict_fine(st, d, B, l, n(l + 1), nchild, x_sel, use_r);
  }
};
}  // namespace

// First level of the V-cycle tail (one workgroup per instance, see k_vcycle_tail): the first
// level l >= 1 with at most `cells` cells (kTailCells unless tuned) such that every level
// l .. L-2 has nx % 4 == 0; L - 1 (only the coarsest solve) when there is none.
static int tail_start(const Layout &Ly, int L, int cells) {
  const long long limit = cells > 0 ? cells : kTailCells;
  int t = L - 1;
  for (int l = L - 2; l >= 1; --l) {
    if (Ly.ln[l] > limit || Ly.lnx[l] % 4 != 0) break;
    t = l;
  }
  return t;
}

// Depth of the fused level kernels for this smoother schedule (Jacobi: nu sweeps; Chebyshev:
// the degree, with one polynomial per side), 0 when there is no fused form or the per-sweep
// kernels are asked for.
static int zm_depth(const InstDesc &H) {
  if (H.vcycle_mode == PLSQR_VCYCLE_PER_SWEEP) return 0;
  if (H.smoother == PLSQR_SMOOTH_JACOBI) return (H.nu_pre >= 1 && H.nu_pre <= 4) ? H.nu_pre : 0;
  return (H.nu_pre == 1 && H.cheb_degree >= 1 && H.cheb_degree <= 4) ? H.cheb_degree : 0;
}

// First level of the LDS-resident tail: the first level l >= 1 with at most `cells` cells
// (kTailCells unless tuned; never more than kTailMaxPer per thread) such that the levels
// l .. coarsest fit its LDS pool; L - 1 (only the coarsest solve) when there is none. Any nx will
// do: the tail works voxel by voxel.
static int tail_start_lds(const Layout &Ly, int L, int cells) {
  const long long limit = std::min<long long>(cells > 0 ? cells : kTailCells,
                                              (long long)kTailMaxPer * kTailBlock);
  int t = L - 1;
  for (int l = L - 2; l >= 1; --l) {
    if (Ly.ln[l] > limit) break;
    if (tail_lds_floats(Ly.ln + l, L - l) > kTailLdsFloats) break;
    t = l;
  }
  return t;
}

// How a V-cycle of this instance runs (levels >= 2): the first tail level, the depth of the
// fused level kernels, and for each level above the tail its fused tile (fz: whether it runs
// fused).
struct VcPlan {
  int t, hz;
  ZmShape shp[kMaxLevels];
  bool fz[kMaxLevels];
};
static VcPlan vcycle_plan(const InstDesc &H, const Layout &Ly) {
  VcPlan P{};
  const int L = H.levels;
  // the fused schedule ends in the LDS-resident tail, the per-sweep one in the tail that keeps
  // its levels in global memory
  const bool fused_mode = H.vcycle_mode != PLSQR_VCYCLE_PER_SWEEP;
  P.t = fused_mode ? tail_start_lds(Ly, L, H.tail_cells) : tail_start(Ly, L, H.tail_cells);
  // levels above the tail whose pre- and post-smoothing each run as one fused launch
  P.hz = zm_depth(H);
  for (int l = 0; l < P.t; ++l) {
    P.shp[l] = zm_shape(Ly.lnx[l], Ly.lny[l], Ly.lnz[l], P.hz > 0 ? P.hz : 1, H.zm_ty, H.zm_zc,
                        H.zm_v);
    P.fz[l] = P.hz > 0 && zm_fits(Ly.lnx[l], P.hz, P.shp[l]);
  }
  // level 0's up kernel writes one alpha partial per block into the instance's partials
  if (P.fz[0] && zm_tiles(Ly.lnx[0], Ly.lny[0], Ly.lnz[0], P.shp[0]) > Ly.nparts) P.fz[0] = false;
  return P;
}

void plan_vcycle(InstDesc &D, const Layout &Ly) {
  for (int l = 0; l < kMaxLevels; ++l) D.zmp[l] = ZmPlan{0, 0, 0, 0};
  D.tail_lds_t = 0;
  if (D.levels < 2) return;
  const VcPlan P = vcycle_plan(D, Ly);
  D.tail_lds_t = P.t;
  for (int l = 0; l < P.t; ++l)
    if (P.fz[l]) D.zmp[l] = ZmPlan{P.shp[l].tx, P.shp[l].ty, P.shp[l].zc, P.shp[l].v};
}

// Whether the beta and alpha finalisers of an inner step run in finaliser blocks of the next
// product's first pass instead of launches of their own: the first pass of a blur product reads
// none of the scalars they write, so the beta finaliser rides in the adjoint product's x pass and
// the alpha finaliser of the V-cycle in the next forward product's x pass (or, after the last
// inner step, in a launch of its own before the per-outer residual); the pending f, w update then
// moves to the forward product's second pass. Needs the fused update, a blur operator whose
// product starts with the four-voxel x pass and has a second pass, and a V-cycle that ends in
// level 0's fused up kernel (its partial count is known before it runs: vcycle_parts).
static bool fin_blocks(const BatchView &bv) {
  const InstDesc &H = *bv.h;
  if (!fused_update(bv) || H.op_kind != PLSQR_OP_BLUR || H.nx % 4 != 0) return false;
  if (H.ny < 2 && H.nz < 2) return false;
  if (H.levels < 2) return false;
  return vcycle_plan(H, *bv.lay).fz[0];
}

// Whether the pending f, w update of an inner step runs in extra workgroups of the next
// V-cycle's tail launch rather than in the forward product (under fin_blocks the tail runs
// after the alpha finaliser that makes the update pending, and before level 0's up kernel
// overwrites v). The tail is one workgroup per instance: at most kTailUpdateVoxels voxels of
// update traffic fit beside it (PLSQR_UPDATE_AUTO).
constexpr long long kTailUpdateVoxels = 1LL << 22;
constexpr int kTailUpdateCUs = 256;   // compute units: one tail-launch workgroup fits a CU
static bool tail_update(const BatchView &bv) {
  const InstDesc &H = *bv.h;
  if (H.update_site == PLSQR_UPDATE_PRODUCT || !fin_blocks(bv) || H.n % 4 != 0) return false;
  return H.update_site == PLSQR_UPDATE_TAIL || (long long)bv.B * H.n <= kTailUpdateVoxels;
}
// update workgroups per instance: the compute units the tails leave free
static int tail_update_parts(const BatchView &bv) {
  return std::max(1, (kTailUpdateCUs - bv.B) / bv.B);
}

// Partials of the alpha reduction that a fused V-cycle leaves: one per block of level 0's up
// kernel.
static int vcycle_parts(const InstDesc &H, const Layout &Ly) {
  const VcPlan P = vcycle_plan(H, Ly);
  return (int)zm_tiles(Ly.lnx[0], Ly.lny[0], Ly.lnz[0], P.shp[0]);
}

// upd_parts > 0: the tail launch also applies the pending f, w update (tail_update).
static int enqueue_vcycle(hipStream_t st, const BatchView &bv, int upd_parts = 0) {
  const InstDesc &H = *bv.h;
  const Layout &Ly = *bv.lay;
  const int L = H.levels;
  InstDesc *const *d = bv.d_descs;
  const int B = bv.B;
  const LevelLaunch K{st, d, B, Ly};
  if (L == 1) {
    launch_coarse_solve(st, d, B);   // exact M^{-1} on a single grid
    return launch_dot_vp(st, d, B, H.n);
  }
  int np = 0;
  const int nu = H.nu_pre;
  const bool fused_mode = H.vcycle_mode != PLSQR_VCYCLE_PER_SWEEP;
  const VcPlan P = vcycle_plan(H, Ly);
  const int t = P.t, hz = P.hz;
  const ZmShape *shp = P.shp;
  const bool *fz = P.fz;
  auto tail = [&]() {
    if (fused_mode) launch_vcycle_tail_lds(st, d, B, t, upd_parts);
    else launch_vcycle_tail(st, d, B, t);
  };
  auto zm = [&](int kind, int l, int want) {
    return launch_zm(st, d, B, kind, hz, l, Ly.lnx[l], Ly.lny[l], Ly.lnz[l], shp[l], want);
  };
  if (H.smoother == PLSQR_SMOOTH_JACOBI) {
    // the first two pre-sweeps run as one kernel; the prolongation runs inside the first
    // post-sweep; every sweep writes the other of the (x, t) pair, ending in x
    const int pre_writes = (nu >= 2) ? nu - 1 : 1;
    const int first_dst = ((pre_writes + nu) % 2) ? LB_X : LB_T;
    int cur_l[kMaxLevels];
    for (int l = 0; l < t; ++l) {
      if (fz[l]) {
        zm(ZM_JAC_DOWN, l, 0);
        continue;
      }
      int cur;
      if (nu >= 2) {
        K.jacobi_first2(l, first_dst, 0);
        cur = first_dst;
        for (int s = 2; s < nu; ++s) {
          K.jacobi(l, 0, cur, other(cur), 0);
          cur = other(cur);
        }
      } else {
        K.jacobi(l, 1, LB_X, first_dst, 0);
        cur = first_dst;
      }
      cur_l[l] = cur;
      K.restrict_to(l, cur, 0);
    }
    tail();
    for (int l = t - 1; l >= 0; --l) {
      if (fz[l]) {
        const int r = zm(ZM_JAC_UP, l, l == 0 ? 1 : 0);
        if (l == 0) np = r;
        continue;
      }
      int cur = cur_l[l];
      const bool last0 = (nu == 1);
      int r = K.jacobi_prolong(l, cur, other(cur), (l == 0 && last0) ? 1 : 0);
      if (l == 0 && last0) np = r;
      cur = other(cur);
      for (int s = 1; s < nu; ++s) {
        const bool last = (s == nu - 1);
        r = K.jacobi(l, 0, cur, other(cur), (l == 0 && last) ? 1 : 0);
        if (l == 0 && last) np = r;
        cur = other(cur);
      }
    }
  } else {
    const int m = H.cheb_degree;
    for (int l = 0; l < t; ++l) {
      if (fz[l]) {
        zm(ZM_CHEB_DOWN, l, 0);
        continue;
      }
      for (int a = 0; a < nu; ++a) {
        int dcur = LB_T;
        int k0 = 0;
        if (a == 0) {
          // start and first step from x = 0 in one kernel
          const bool last = (m == 1);
          K.cheb_first(l, last ? 1 : 0, LB_T);
          k0 = 1;
        } else {
          K.cheb_start(l, 0, LB_T);
        }
        for (int k = k0; k < m; ++k) {
          const bool last = (k == m - 1);
          const bool upd = !last || (a == nu - 1);
          const int dn = other_d(dcur);
          K.cheb_step(l, 0, upd ? 1 : 0, last ? 1 : 0, dcur, dn, k, 0, 0);
          dcur = dn;
        }
      }
      K.restrict_to(l, LB_X, 1);
    }
    tail();
    for (int l = t - 1; l >= 0; --l) {
      if (fz[l]) {
        const int r = zm(ZM_CHEB_UP, l, l == 0 ? 1 : 0);
        if (l == 0) np = r;
        continue;
      }
      for (int a = 0; a < nu; ++a) {
        if (a == 0)
          K.cheb_start_prolong(l, LB_T);
        else
          K.cheb_start(l, 0, LB_T);
        int dcur = LB_T;
        for (int k = 0; k < m; ++k) {
          const bool last = (k == m - 1);
          const int dn = other_d(dcur);
          const bool want = (l == 0 && a == nu - 1 && last);
          const int r = K.cheb_step(l, 0, last ? 0 : 1, last ? 1 : 0, dcur, dn, k, want ? 1 : 0,
                                    (a == 0 && k == 0) ? 1 : 0);
          if (want) np = r;
          dcur = dn;
        }
      }
    }
  }
  return np;
}

// ---------------------------------------------------------------------------------
// phases
// ---------------------------------------------------------------------------------
void enqueue_request_begin(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  launch_request_begin(st, bv.d_descs, bv.B, H.n);
  const int np = launch_diffusivity(st, bv.d_descs, bv.B, H.n, 1);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_PENALTY);
}

void enqueue_outer_setup(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  const Layout &Ly = *bv.lay;
  launch_outer_begin(st, bv.d_descs, bv.B);
  launch_level0_dinv(st, bv.d_descs, bv.B, H.n);
  for (int l = 0; l + 1 < H.levels; ++l) {
    launch_coarsen(st, bv.d_descs, bv.B, l, Ly.ln[l + 1]);
    launch_level_dinv(st, bv.d_descs, bv.B, l + 1, Ly.ln[l + 1]);
  }
  launch_coarse_factor(st, bv.d_descs, bv.B);
}

void enqueue_mlsqr_init(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  int np = launch_copy_g_u(st, bv.d_descs, bv.B, H.m);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_BETA_INIT);
  enqueue_adjoint(st, bv, EPI_ADJ_INIT);
  np = enqueue_vcycle(st, bv);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_ALPHA_INIT);
  launch_init_wf(st, bv.d_descs, bv.B, H.n);
  if (H.stop_flags & PLSQR_FLAG_STOP_S4) launch_s4_begin(st, bv.d_descs, bv.B, H.m);
  if (H.n_tau > 0) launch_basis_store(st, bv.d_descs, bv.B, H.n);
}

// After the f/w update: the S4 residual of the new iterate, and the stop test.
static void enqueue_s4(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  if (!(H.stop_flags & PLSQR_FLAG_STOP_S4)) return;
  const int np = launch_s4_step(st, bv.d_descs, bv.B, H.m);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_S4);
}

// The update step after the alpha reduction: f, w (unless the next forward product applies it),
// the S4 recurrence, the stored basis.
static void enqueue_update(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  if (!fused_update(bv)) launch_update_fw(st, bv.d_descs, bv.B, H.n);
  enqueue_s4(st, bv);
  if (H.n_tau > 0) launch_basis_store(st, bv.d_descs, bv.B, H.n);
}

// Whether enqueue_update enqueues nothing: the update rides on the next forward product, and
// there is no S4 recurrence or stored basis (fused_update requires both).
static bool update_fused_whole(const BatchView &bv) { return fused_update(bv); }

// The products of an inner step with the beta finaliser between them; under fin_blocks the
// alpha finaliser of the last V-cycle (if one is pending) rides in the forward product and beta
// in the adjoint product, and the forward product applies the pending update unless the
// V-cycle's tail does (tail_update).
static void enqueue_inner_products(hipStream_t st, const BatchView &bv) {
  if (fin_blocks(bv)) {
    const bool tu = tail_update(bv);
    const int nb = enqueue_forward(st, bv, V_V, EPI_FWD, !tu, tu ? FIN_ALPHA_PEND_T : FIN_ALPHA_PEND,
                                   vcycle_parts(*bv.h, *bv.lay));
    enqueue_adjoint(st, bv, EPI_ADJ, tu ? FIN_BETA_PEND_T : FIN_BETA_PEND, nb);
    return;
  }
  const int np = enqueue_forward(st, bv, V_V, EPI_FWD, true);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_BETA);
  enqueue_adjoint(st, bv, EPI_ADJ);
}

// The V-cycle of an inner step and the alpha finaliser (under fin_blocks its partials wait for
// the next forward product).
static void enqueue_inner_vcycle(hipStream_t st, const BatchView &bv) {
  const int np = enqueue_vcycle(st, bv, tail_update(bv) ? tail_update_parts(bv) : 0);
  if (!fin_blocks(bv)) launch_finalize(st, bv.d_descs, bv.B, np, FIN_ALPHA);
}

void enqueue_inner(hipStream_t st, const BatchView &bv) {
  enqueue_inner_products(st, bv);
  enqueue_inner_vcycle(st, bv);
  enqueue_update(st, bv);
}

// ---------------------------------------------------------------------------------
// inner steps of instances of different grids in shared launches
// ---------------------------------------------------------------------------------
bool ragged_ok(const InstDesc &H, const Layout &Ly) {
  if (H.op_kind != PLSQR_OP_BLUR || H.nz < 2 || H.ny < 2 || H.nx % 4 != 0) return false;
  if (H.n_tau > 0 || (H.stop_flags & PLSQR_FLAG_STOP_S4) || H.levels < 2) return false;
  if (H.vcycle_mode == PLSQR_VCYCLE_PER_SWEEP) return false;
  const VcPlan P = vcycle_plan(H, Ly);
  for (int l = 0; l < P.t; ++l)
    if (!P.fz[l]) return false;
  return true;
}

namespace {
// A ragged map over the instances `who` (indices into the batch), count(i) blocks each, every
// range starting at a multiple of 8.
template <class F>
Rag rag_over(const std::vector<int> &who, F count) {
  Rag r{};
  r.n = (int)who.size();
  int off = 0;
  for (int k = 0; k < r.n; ++k) {
    r.inst[k] = who[k];
    r.first[k] = off;
    r.count[k] = count(who[k]);
    off = (off + r.count[k] + 7) / 8 * 8;
  }
  return r;
}
}  // namespace

void enqueue_inner_ragged(hipStream_t st, const RagBatch &rb) {
  const int B = rb.B;
  InstDesc *const *d = rb.d_descs;
  const InstDesc &H0 = *rb.h[0];
  std::vector<int> all(B);
  for (int i = 0; i < B; ++i) all[i] = i;
  auto h = [&](int i) -> const InstDesc & { return *rb.h[i]; };
  std::vector<VcPlan> P(B);
  int T = 0;
  for (int i = 0; i < B; ++i) {
    P[i] = vcycle_plan(h(i), *rb.lay[i]);
    T = std::max(T, P[i].t);
  }
  // blur product: x, y, z passes, the last with the epilogue; the x pass carries a finaliser
  // block per instance for `fin` on the partial counts fnp (ragged_ok implies fin_blocks for
  // every instance), the forward product's y pass applies the pending update; returns the last
  // pass's map
  auto blur = [&](int src, int adj, int epi, int fin, const Rag &fnp) {
    const int em = with_mask(H0, epi);
    const int e_mid = EPI_STORE | (em & (EPI_MASK_INNER | EPI_MASK_OUTER));
    const Rag rx = rag_over(all, [&](int i) { return blur_x_blocks(h(i).n, h(i).nx, H0.blur_xgroups) + 1; });
    launch_blur_x(st, d, B, H0.n, H0.nx, src, V_TMP1, adj, e_mid, H0.blur_xgroups, rx, 0, fin, 0,
                  fnp);
    const Rag ry = rag_over(all, [&](int i) {
      return blur_axis_blocks(h(i).nx, h(i).ny, h(i).nz, 1, H0.blur_window);
    });
    launch_blur_axis(st, d, B, H0.nx, H0.ny, H0.nz, 1, V_TMP1, V_TMP2, adj, e_mid, H0.blur_window, ry,
                     (adj == 0 && epi == EPI_FWD) ? 1 : 0);
    const Rag rz = rag_over(all, [&](int i) {
      return blur_axis_blocks(h(i).nx, h(i).ny, h(i).nz, 2, H0.blur_window);
    });
    launch_blur_axis(st, d, B, H0.nx, H0.ny, H0.nz, 2, V_TMP2, V_TMP2, adj, em, H0.blur_window, rz);
    return rz;
  };
  // the pending alpha finaliser of each instance's last V-cycle: one partial per block of its
  // level-0 up kernel
  const Rag na = rag_over(all, [&](int i) {
    const Layout &Ly = *rb.lay[i];
    return (int)zm_tiles(Ly.lnx[0], Ly.lny[0], Ly.lnz[0], P[i].shp[0]);
  });
  const Rag nb = blur(V_V, 0, EPI_FWD, FIN_ALPHA_PEND, na);
  blur(V_U, 1, EPI_ADJ, FIN_BETA_PEND, nb);

  // V-cycle by depth from the finest level: the down halves of depth 0, 1, .. (an instance takes
  // part while the depth is above its tail), every instance's LDS-resident tail in one launch,
  // then the up halves back to depth 0; instances of one depth with different voxels per
  // thread take one launch each; level 0's partials of v.p wait for the next forward product
  const int H = P[0].hz;
  const bool jac = H0.smoother == PLSQR_SMOOTH_JACOBI;
  auto depth = [&](int dd, bool down) {
    for (int v : {4, 1}) {
      std::vector<int> who;
      for (int i = 0; i < B; ++i)
        if (P[i].t > dd && P[i].shp[dd].v == v) who.push_back(i);
      if (who.empty()) continue;
      int threads = 0;
      size_t lds = 0;
      for (int i : who) {
        threads = std::max(threads, zm_threads(P[i].shp[dd], H));
        lds = std::max(lds, zm_lds_bytes(H, P[i].shp[dd], down));
      }
      const Rag rg = rag_over(who, [&](int i) {
        const Layout &Ly = *rb.lay[i];
        return (int)zm_tiles(Ly.lnx[dd], Ly.lny[dd], Ly.lnz[dd], P[i].shp[dd]);
      });
      const int kind = down ? (jac ? ZM_JAC_DOWN : ZM_CHEB_DOWN) : (jac ? ZM_JAC_UP : ZM_CHEB_UP);
      const int want = (!down && dd == 0) ? 1 : 0;
      launch_zm_ragged(st, d, kind, H, dd, v, threads, lds, rg, want);
    }
  };
  for (int dd = 0; dd < T; ++dd) depth(dd, true);
  launch_vcycle_tail_lds(st, d, B, -1);
  for (int dd = T - 1; dd >= 0; --dd) depth(dd, false);
}

void enqueue_outer_end(hipStream_t st, const BatchView &bv) {
  const InstDesc &H = *bv.h;
  // the last inner step's alpha finaliser, left pending (fin_blocks), and its update, left
  // pending (fused_update)
  if (fin_blocks(bv))
    launch_finalize(st, bv.d_descs, bv.B, vcycle_parts(H, *bv.lay),
                    tail_update(bv) ? FIN_ALPHA_PEND_T : FIN_ALPHA_PEND);
  if (fused_update(bv)) launch_update_fw(st, bv.d_descs, bv.B, H.n, kNoRag, 1);
  int np = enqueue_forward(st, bv, V_F, EPI_RESID);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_RESID);
  np = launch_diffusivity(st, bv.d_descs, bv.B, H.n, 1);
  launch_finalize(st, bv.d_descs, bv.B, np, FIN_PENALTY);
}

void enqueue_request_end(hipStream_t st, const BatchView &bv) {
  if (bv.h->n_tau > 0) launch_tau_finish(st, bv.d_descs, bv.B, bv.h->n, bv.h->n_tau);
  launch_copy_out(st, bv.d_descs, bv.B, bv.h->n);
}

GraphCache::~GraphCache() {
  for (hipGraphExec_t e : execs) hipGraphExecDestroy(e);
  if (cap) hipStreamDestroy(cap);
}

// Capture `body` (kernel launches only) into an executable graph.
template <class F>
static hipGraphExec_t capture_graph(hipStream_t cap, F body) {
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  body(cap);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(cap, &g) != hipSuccess || !g) return nullptr;
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e == hipSuccess ? ex : nullptr;
}

// Inner steps per graph on the untimed path: consecutive launches of one graph start about 9 us
// apart on MI355X (against well under 1 us between the kernels inside a graph), so several steps
// go into one graph, and a second graph holds the rest of an outer step's inner count.
constexpr int kStepsPerGraph = 8;

// The inner iteration through graphs. With product timing the two products stay eager
// (each bracketed by events on the engine stream) and only the kernels after the adjoint
// product (V-cycle, alpha reduction and rotations, update) replay as a graph; otherwise
// min(inner, kStepsPerGraph) whole iterations form one graph (execs[0]) and the remainder of
// inner another (execs[1], when there is one). Returns false if capture is unavailable.
static bool prepare_inner_graphs(const BatchView &bv, GraphCache &gc, int inner) {
  if (!gc.execs.empty()) return true;
  if (!gc.cap && hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking) != hipSuccess) return false;
  BatchView quiet = bv;
  quiet.prod_events = nullptr;
  quiet.adj_events = nullptr;
  const bool timed = bv.prod_events != nullptr;
  auto vcycle_part = [&](hipStream_t s) { enqueue_inner_vcycle(s, quiet); };
  auto update_part = [&](hipStream_t s) { enqueue_update(s, quiet); };
  std::vector<hipGraphExec_t> ex;
  if (bv.vcycle_events) {
    // phases timed: the V-cycle part and the update part replay as two graphs (the update part
    // is empty when the next forward product applies the update)
    ex.push_back(capture_graph(gc.cap, vcycle_part));
    if (!update_fused_whole(bv)) ex.push_back(capture_graph(gc.cap, update_part));
  } else if (timed) {
    ex.push_back(capture_graph(gc.cap, [&](hipStream_t s) {
      vcycle_part(s);
      update_part(s);
    }));
  } else {
    const int k = std::min(inner, kStepsPerGraph), rest = inner % k;
    ex.push_back(capture_graph(gc.cap, [&](hipStream_t s) {
      for (int i = 0; i < k; ++i) enqueue_inner(s, quiet);
    }));
    if (rest)
      ex.push_back(capture_graph(gc.cap, [&](hipStream_t s) {
        for (int i = 0; i < rest; ++i) enqueue_inner(s, quiet);
      }));
  }
  for (hipGraphExec_t e : ex)
    if (!e) {
      for (hipGraphExec_t f : ex)
        if (f) hipGraphExecDestroy(f);
      return false;
    }
  gc.execs = ex;
  return true;
}

// Events around one phase when its list is given.
template <class F>
static void timed_phase(hipStream_t st, EventList *ev, F body) {
  hipEvent_t a = nullptr;
  time_begin(st, ev, &a);
  body();
  time_end(st, ev, a);
}

void enqueue_whole_solve(hipStream_t st, const BatchView &bv, int outer, int inner,
                         GraphCache *graphs) {
  const bool use_graphs = graphs && prepare_inner_graphs(bv, *graphs, inner);
  const bool timed = bv.prod_events != nullptr;
  const bool phases = bv.vcycle_events != nullptr;
  timed_phase(st, bv.setup_events, [&] { enqueue_request_begin(st, bv); });
  for (int k = 1; k <= outer; ++k) {
    timed_phase(st, bv.setup_events, [&] {
      enqueue_outer_setup(st, bv);
      enqueue_mlsqr_init(st, bv);
    });
    if (!timed && use_graphs) {   // (phase timing implies product timing)
      const int g = std::min(inner, kStepsPerGraph);
      for (int i = 0; i + g <= inner; i += g) hipGraphLaunch(graphs->execs[0], st);
      if (inner % g) hipGraphLaunch(graphs->execs[1], st);
      timed_phase(st, bv.diag_events, [&] { enqueue_outer_end(st, bv); });
      continue;
    }
    for (int i = 0; i < inner; ++i) {
      if (!timed) {
        enqueue_inner(st, bv);
        continue;
      }
      enqueue_inner_products(st, bv);
      if (phases) {
        timed_phase(st, bv.vcycle_events, [&] {
          if (use_graphs) hipGraphLaunch(graphs->execs[0], st);
          else enqueue_inner_vcycle(st, bv);
        });
        timed_phase(st, bv.update_events, [&] {
          if (update_fused_whole(bv)) return;
          if (use_graphs) hipGraphLaunch(graphs->execs[1], st);
          else enqueue_update(st, bv);
        });
      } else if (use_graphs) {
        hipGraphLaunch(graphs->execs[0], st);
      } else {
        enqueue_inner_vcycle(st, bv);
        enqueue_update(st, bv);
      }
    }
    timed_phase(st, bv.diag_events, [&] { enqueue_outer_end(st, bv); });
  }
  timed_phase(st, bv.diag_events, [&] { enqueue_request_end(st, bv); });
}

}  // namespace plsqr
