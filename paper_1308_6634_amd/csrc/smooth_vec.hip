// Four-voxel-per-thread forms of the multigrid level kernels (smoothers, fused prolongation,
// restriction). They compute the same values as the one-voxel kernels in kernels.hip, in the
// same order of floating-point operations per voxel, but every thread owns four consecutive
// voxels of one x-row, so the level vectors move as 16-byte loads and stores. They apply to a
// level whose nx is a multiple of 4 (then every row starts on a 16-byte boundary: the level
// buffers are 256-byte aligned); the V-cycle driver falls back to the one-voxel
// kernels otherwise.
//
// Multigrid V-cycle with Galerkin coarse operators, damped Jacobi and Chebyshev smoothing: the
// fixed approximate inverse of the priorconditioner M (section 4.2).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

__device__ __forceinline__ V4 add4(const V4 &a, const V4 &b) {
  V4 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r.v[e] = a.v[e] + b.v[e];
  return r;
}
__device__ __forceinline__ V4 sub4(const V4 &a, const V4 &b) {
  V4 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r.v[e] = a.v[e] - b.v[e];
  return r;
}
__device__ __forceinline__ double dot4(const V4 &a, const V4 &b) {
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) s += (double)a.v[e] * (double)b.v[e];
  return s;
}

// x + P e on the four voxels of row q (coord cq, cq.x % 4 == 0): voxels 0,1 share one coarse
// parent, voxels 2,3 the next one along x.
__device__ __forceinline__ V4 prolonged4(const LevelDesc &F, const LevelDesc &Cl,
                                         const float *__restrict__ x, const float *__restrict__ e,
                                         long long q, Coord cq) {
  const long long p = parent_of(F, Cl, cq);
  const float e0 = e[p], e1 = e[p + 1];
  V4 r = ld4(x + q);
  r.v[0] += e0;
  r.v[1] += e0;
  r.v[2] += e1;
  r.v[3] += e1;
  return r;
}

__device__ __forceinline__ void write_dot(const InstDesc &D, double dot) {
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

}  // namespace

// ------------------------------------------------------------------------------------
// Per-row bodies: the work of one thread (four voxels j..j+3 of one x-row, j % 4 == 0) in
// each level kernel. They return the thread's part of the sum x.b where the kernel reduces it.
// The standalone kernels run one body per thread over the whole grid; the V-cycle tail kernel
// below runs them in loops inside one workgroup.
// ------------------------------------------------------------------------------------
namespace {

// Damped Jacobi sweep dst = src + omega D^{-1} (b - A src)  (first: src = 0).
__device__ __forceinline__ double body_jacobi(const InstDesc &D, const LevelDesc &L, int l,
                                              long long j, int first, int src_sel, int dst_sel,
                                              int want_dot) {
  const V4 b = ld4(L.b + j);
  V4 xn;
  if (first) {
    const V4 dv = ld4(L.dinv + j);
#pragma unroll
    for (int e = 0; e < 4; ++e) xn.v[e] = sld(D.omega) * dv.v[e] * b.v[e];
  } else {
    const float *__restrict__ src = lvbuf(L, src_sel);
    const Coord c = coord_of(j, L.nx, L.ny);
    auto X4 = [&](long long q, Coord) { return ld4(src + q); };
    auto X1 = [&](long long q, Coord) { return src[q]; };
    const V4 xc = ld4(src + j);
    V4 dv;
    const V4 ax = stencil4(D, L, l, j, c, xc, X4, X1, dv);
#pragma unroll
    for (int e = 0; e < 4; ++e) xn.v[e] = xc.v[e] + sld(D.omega) * dv.v[e] * (b.v[e] - ax.v[e]);
  }
  st4(lvbuf(L, dst_sel) + j, xn);
  return want_dot ? dot4(xn, b) : 0.0;
}

// First two damped Jacobi sweeps from x = 0: x1 = omega D^{-1} b formed on the fly (also at
// the neighbours), dst = x1 + omega D^{-1} (b - A x1).
__device__ __forceinline__ double body_jacobi_first2(const InstDesc &D, const LevelDesc &L, int l,
                                                     long long j, int dst_sel, int want_dot) {
  const float *__restrict__ b = L.b;
  const float *__restrict__ dinv = L.dinv;
  const float om = sld(D.omega);
  const Coord c = coord_of(j, L.nx, L.ny);
  auto X4 = [&](long long q, Coord) {
    const V4 bb = ld4(b + q), dd = ld4(dinv + q);
    V4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r.v[e] = om * dd.v[e] * bb.v[e];
    return r;
  };
  auto X1 = [&](long long q, Coord) { return om * dinv[q] * b[q]; };
  const V4 bj = ld4(b + j), dj = ld4(dinv + j);
  const V4 xc = X4(j, c);
  V4 unused;
  const V4 ax = stencil4(D, L, l, j, c, xc, X4, X1, unused);
  V4 xn;
#pragma unroll
  for (int e = 0; e < 4; ++e) xn.v[e] = xc.v[e] + om * dj.v[e] * (bj.v[e] - ax.v[e]);
  st4(lvbuf(L, dst_sel) + j, xn);
  return want_dot ? dot4(xn, bj) : 0.0;
}

// Prolongation fused into the first post-smoothing Jacobi sweep: x' = x + P e (on the fly at
// the neighbours too), dst = x' + omega D^{-1} (b - A x').
__device__ __forceinline__ double body_jacobi_prolong(const InstDesc &D, const LevelDesc &L,
                                                      const LevelDesc &Cl, int l, long long j,
                                                      int src_sel, int dst_sel, int want_dot) {
  const float *__restrict__ x = lvbuf(L, src_sel);
  const float *__restrict__ ce = Cl.x;
  const Coord c = coord_of(j, L.nx, L.ny);
  auto X4 = [&](long long q, Coord cq) { return prolonged4(L, Cl, x, ce, q, cq); };
  auto X1 = [&](long long q, Coord cq) { return x[q] + ce[parent_of(L, Cl, cq)]; };
  const V4 xc = X4(j, c);
  V4 unused;
  const V4 ax = stencil4(D, L, l, j, c, xc, X4, X1, unused);
  const V4 bj = ld4(L.b + j), dj = ld4(L.dinv + j);
  V4 xn;
#pragma unroll
  for (int e = 0; e < 4; ++e) xn.v[e] = xc.v[e] + sld(D.omega) * dj.v[e] * (bj.v[e] - ax.v[e]);
  st4(lvbuf(L, dst_sel) + j, xn);
  return want_dot ? dot4(xn, bj) : 0.0;
}

// Chebyshev recurrence coefficients of step `step`: rho_0 = 1/sigma,
// rho_{k+1} = 1/(2 sigma - rho_k); d' = rho_{k+1} rho_k d + 2 rho_{k+1}/delta D^{-1} r.
__device__ __forceinline__ void cheb_coefs(const InstDesc &D, int step, float &c_dd, float &c_dr) {
  double rho = 1.0 / sld(D.cheb_sigma);
  for (int i = 0; i < step; ++i) rho = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  const double rho_next = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  c_dd = (float)(rho_next * rho);
  c_dr = (float)(2.0 * rho_next / sld(D.cheb_delta));
}

// Chebyshev pre-smoothing start fused with its first step (x = 0): d0 = D^{-1} b / theta on
// the fly, x1 = d0, r1 = b - A d0, and (unless the polynomial has degree 1) d1 -> dn_sel.
__device__ __forceinline__ void body_cheb_first(const InstDesc &D, const LevelDesc &L, int l,
                                                long long j, int last, int dn_sel, float c_dd,
                                                float c_dr) {
  const float ith = (float)(1.0 / sld(D.cheb_theta));
  const float *__restrict__ b = L.b;
  const float *__restrict__ dinv = L.dinv;
  const Coord c = coord_of(j, L.nx, L.ny);
  auto X4 = [&](long long q, Coord) {
    const V4 bb = ld4(b + q), dd = ld4(dinv + q);
    V4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r.v[e] = ith * dd.v[e] * bb.v[e];
    return r;
  };
  auto X1 = [&](long long q, Coord) { return ith * dinv[q] * b[q]; };
  const V4 bj = ld4(b + j), dj = ld4(dinv + j);
  const V4 d0 = X4(j, c);
  st4(L.x + j, d0);
  V4 unused;
  const V4 r = sub4(bj, stencil4(D, L, l, j, c, d0, X4, X1, unused));
  st4(L.r + j, r);
  if (!last) {
    V4 dn;
#pragma unroll
    for (int e = 0; e < 4; ++e) dn.v[e] = c_dd * d0.v[e] + c_dr * dj.v[e] * r.v[e];
    st4(lvbuf(L, dn_sel) + j, dn);
  }
}

// Chebyshev post-smoothing start fused with the prolongation: r = b - A x' with x' = x + P e
// formed on the fly (x is left alone: other threads still read it; the first step adds P e
// pointwise), d = D^{-1} r / theta -> d_sel.
__device__ __forceinline__ void body_cheb_start_prolong(const InstDesc &D, const LevelDesc &L,
                                                        const LevelDesc &Cl, int l, long long j,
                                                        int d_sel) {
  const float *__restrict__ x = L.x;
  const float *__restrict__ ce = Cl.x;
  const Coord c = coord_of(j, L.nx, L.ny);
  auto X4 = [&](long long q, Coord cq) { return prolonged4(L, Cl, x, ce, q, cq); };
  auto X1 = [&](long long q, Coord cq) { return x[q] + ce[parent_of(L, Cl, cq)]; };
  const V4 xc = X4(j, c);
  V4 unused;
  const V4 r = sub4(ld4(L.b + j), stencil4(D, L, l, j, c, xc, X4, X1, unused));
  st4(L.r + j, r);
  const V4 dj = ld4(L.dinv + j);
  const float ith = (float)(1.0 / sld(D.cheb_theta));
  V4 d;
#pragma unroll
  for (int e = 0; e < 4; ++e) d.v[e] = ith * dj.v[e] * r.v[e];
  st4(lvbuf(L, d_sel) + j, d);
}

// Chebyshev start: r = b - A x (or r = b when x = 0), d = D^{-1} r / theta -> d_sel.
__device__ __forceinline__ void body_cheb_start(const InstDesc &D, const LevelDesc &L, int l,
                                                long long j, int zero_x, int d_sel) {
  V4 r = ld4(L.b + j);
  V4 dv;
  if (!zero_x) {
    const float *__restrict__ x = L.x;
    const Coord c = coord_of(j, L.nx, L.ny);
    auto X4 = [&](long long q, Coord) { return ld4(x + q); };
    auto X1 = [&](long long q, Coord) { return x[q]; };
    r = sub4(r, stencil4(D, L, l, j, c, ld4(x + j), X4, X1, dv));
  } else {
    dv = ld4(L.dinv + j);
  }
  st4(L.r + j, r);
  const float ith = (float)(1.0 / sld(D.cheb_theta));
  V4 d;
#pragma unroll
  for (int e = 0; e < 4; ++e) d.v[e] = ith * dv.v[e] * r.v[e];
  st4(lvbuf(L, d_sel) + j, d);
}

// One Chebyshev step: x += d (x = d when set_x; plus P e when add_prolong); r -= A d (if
// update_r); d' = c_dd d + c_dr D^{-1} r (if !last), d read from d_sel, d' written to dn_sel.
// With want_dot, the part of sum x_j b_j after the update.
__device__ __forceinline__ double body_cheb_step(const InstDesc &D, const LevelDesc &L,
                                                 const LevelDesc &Cl, int l, long long j,
                                                 int set_x, int update_r, int last, int d_sel,
                                                 int dn_sel, int want_dot, int add_prolong,
                                                 float c_dd, float c_dr) {
  const float *__restrict__ d = lvbuf(L, d_sel);
  const Coord c = coord_of(j, L.nx, L.ny);
  const V4 dj = ld4(d + j);
  V4 xo = {};
  if (!set_x) xo = ld4(L.x + j);
  if (add_prolong) {
    const long long p = parent_of(L, Cl, c);
    const float e0 = Cl.x[p], e1 = Cl.x[p + 1];
    xo.v[0] += e0;
    xo.v[1] += e0;
    xo.v[2] += e1;
    xo.v[3] += e1;
  }
  const V4 xn = add4(xo, dj);
  st4(L.x + j, xn);
  const double dot = want_dot ? dot4(xn, ld4(L.b + j)) : 0.0;
  if (update_r) {
    auto X4 = [&](long long q, Coord) { return ld4(d + q); };
    auto X1 = [&](long long q, Coord) { return d[q]; };
    V4 dv;
    const V4 r = sub4(ld4(L.r + j), stencil4(D, L, l, j, c, dj, X4, X1, dv));
    st4(L.r + j, r);
    if (!last) {
      V4 dn;
#pragma unroll
      for (int e = 0; e < 4; ++e) dn.v[e] = c_dd * dj.v[e] + c_dr * dv.v[e] * r.v[e];
      st4(lvbuf(L, dn_sel) + j, dn);
    }
  }
  return dot;
}

// Restriction of the residual: b_{l+1}[J] = sum over the children j of J of (b - A_l x)_j, or
// of a stored residual r_l when use_r, for the pair of x-adjacent coarse cells J, J+1 (J even):
// their children are four consecutive fine voxels in each of the 2 (2D) or 4 (3D) fine rows.
__device__ __forceinline__ void body_restrict(const InstDesc &D, const LevelDesc &F,
                                              const LevelDesc &Cl, int l, long long J, int x_sel,
                                              int use_r) {
  const Coord cc = coord_of(J, Cl.nx, Cl.ny);
  const int cz = (F.nz > 1) ? 2 : 1;
  const float *__restrict__ x = lvbuf(F, x_sel);
  auto X4 = [&](long long q, Coord) { return ld4(x + q); };
  auto X1 = [&](long long q, Coord) { return x[q]; };
  float s0 = 0.f, s1 = 0.f;
  for (int dz = 0; dz < cz; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      Coord fc;
      fc.x = 2 * cc.x;
      fc.y = 2 * cc.y + dy;
      fc.z = cz * cc.z + dz;
      const long long jf = fc.x + (long long)F.nx * (fc.y + (long long)F.ny * fc.z);
      V4 v;
      if (use_r) {
        v = ld4(F.r + jf);
      } else {
        V4 unused;
        v = sub4(ld4(F.b + jf), stencil4(D, F, l, jf, fc, ld4(x + jf), X4, X1, unused));
      }
      s0 += v.v[0];
      s0 += v.v[1];
      s1 += v.v[2];
      s1 += v.v[3];
    }
  *reinterpret_cast<float2 *>(Cl.b + J) = make_float2(s0, s1);
}

}  // namespace

// ------------------------------------------------------------------------------------
// One-pass kernels (one body per thread)
// ------------------------------------------------------------------------------------
// the z-neighbour planes of a block's rows belong to blocks nx*ny/1024 tiles away: xcd_tile
// keeps them on the same XCD
#define ROW_INDEX() (4 * (xcd_tile() * kBlock + threadIdx.x))

__global__ void __launch_bounds__(kBlock) k_jacobi4(InstDesc *const *descs, int l, int first,
                                                   int src_sel, int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = ROW_INDEX();
  double dot = 0.0;
  if (j < L.n) dot = body_jacobi(D, L, l, j, first, src_sel, dst_sel, want_dot);
  if (want_dot) write_dot(D, dot);
}

__global__ void __launch_bounds__(kBlock) k_jacobi_first2_4(InstDesc *const *descs, int l,
                                                           int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = ROW_INDEX();
  double dot = 0.0;
  if (j < L.n) dot = body_jacobi_first2(D, L, l, j, dst_sel, want_dot);
  if (want_dot) write_dot(D, dot);
}

__global__ void __launch_bounds__(kBlock) k_jacobi_prolong4(InstDesc *const *descs, int l,
                                                           int src_sel, int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l), Cl = level_of(D, l + 1);
  const long long j = ROW_INDEX();
  double dot = 0.0;
  if (j < L.n) dot = body_jacobi_prolong(D, L, Cl, l, j, src_sel, dst_sel, want_dot);
  if (want_dot) write_dot(D, dot);
}

__global__ void __launch_bounds__(kBlock) k_cheb_first4(InstDesc *const *descs, int l, int last,
                                                       int dn_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = ROW_INDEX();
  if (j >= L.n) return;
  float c_dd, c_dr;
  cheb_coefs(D, 0, c_dd, c_dr);
  body_cheb_first(D, L, l, j, last, dn_sel, c_dd, c_dr);
}

__global__ void __launch_bounds__(kBlock) k_cheb_start_prolong4(InstDesc *const *descs, int l,
                                                               int d_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l), Cl = level_of(D, l + 1);
  const long long j = ROW_INDEX();
  if (j < L.n) body_cheb_start_prolong(D, L, Cl, l, j, d_sel);
}

__global__ void __launch_bounds__(kBlock) k_cheb_start4(InstDesc *const *descs, int l, int zero_x,
                                                       int d_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = ROW_INDEX();
  if (j < L.n) body_cheb_start(D, L, l, j, zero_x, d_sel);
}

__global__ void __launch_bounds__(kBlock) k_cheb_step4(InstDesc *const *descs, int l, int set_x,
                                                      int update_r, int last, int d_sel,
                                                      int dn_sel, int step, int want_dot,
                                                      int add_prolong) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l), Cl = level_of(D, l + 1);
  const long long j = ROW_INDEX();
  float c_dd, c_dr;
  cheb_coefs(D, step, c_dd, c_dr);
  double dot = 0.0;
  if (j < L.n)
    dot = body_cheb_step(D, L, Cl, l, j, set_x, update_r, last, d_sel, dn_sel, want_dot,
                         add_prolong, c_dd, c_dr);
  if (want_dot) write_dot(D, dot);
}

__global__ void __launch_bounds__(kBlock) k_restrict4(InstDesc *const *descs, int l, int x_sel,
                                                     int use_r) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc F = level_of(D, l), Cl = level_of(D, l + 1);
  const long long J = 2 * ((long long)blockIdx.x * kBlock + threadIdx.x);
  if (J < Cl.n) body_restrict(D, F, Cl, l, J, x_sel, use_r);
}

// ------------------------------------------------------------------------------------
// V-cycle tail: every level from `t` (>= 1) down to the coarsest and back up, in one
// workgroup of kTailBlock threads per instance. On the small coarse levels the one-pass
// kernels are bound by launch and dependency latency rather than by memory; here each pass
// is a loop over the level's rows followed by a workgroup barrier (which also orders the
// workgroup's global-memory writes before the next pass's reads), with the same per-row
// arithmetic as the one-pass kernels. Input: b on level t; output: x on level t (restricted
// from and prolongated to level t - 1 by the one-pass kernels). Every level t .. L-2 has
// nx % 4 == 0. The coarsest solve x = A_c^{-1} b splits each row of the FP64 inverse over a
// group of lanes (a power of two) and sums the lane parts with shuffles.
// ------------------------------------------------------------------------------------
namespace {

template <class F>
__device__ __forceinline__ void tail_rows(long long n, F body) {
  for (long long g = threadIdx.x; 4 * g < n; g += kTailBlock) body(4 * g);
  __syncthreads();
}

__device__ __forceinline__ int other_x(int s) { return s == LB_X ? LB_T : LB_X; }
__device__ __forceinline__ int other_d(int s) { return s == LB_T ? LB_S : LB_T; }

__device__ void tail_coarse_solve(const InstDesc &D, const LevelDesc &L, double *bs) {
  const int n = (int)L.n;
  const double *__restrict__ Ai = sld(D.cfac) + (long long)n * n * 2;
  for (int i = threadIdx.x; i < n; i += kTailBlock) bs[i] = (double)L.b[i];
  __syncthreads();
  int g = 1;   // lanes per row: the largest power of two <= min(64, kTailBlock / n)
  while (2 * g <= 64 && 2 * g * n <= kTailBlock) g *= 2;
  const int s = threadIdx.x % g;
  const int rows_per_pass = kTailBlock / g;
  for (int i0 = 0; i0 < n; i0 += rows_per_pass) {
    const int i = i0 + (int)threadIdx.x / g;
    double acc = 0.0;
    if (i < n)
      for (int j = s; j < n; j += g) acc += Ai[(long long)j * n + i] * bs[j];
    for (int o = 1; o < g; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (i < n && s == 0) L.x[i] = (float)acc;
  }
  __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(kTailBlock) k_vcycle_tail(InstDesc *const *descs, int t) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  __shared__ double bs[PLSQR_MAX_COARSE];
  const int Lv = sld(D.levels);
  const int nu = sld(D.nu_pre);
  if (sld(D.smoother) == PLSQR_SMOOTH_JACOBI) {
    const int pre_writes = (nu >= 2) ? nu - 1 : 1;
    const int first_dst = ((pre_writes + nu) % 2) ? LB_X : LB_T;
    unsigned cur_is_x = 0;   // bit l: level l's pre-smoothed iterate is in x (else in t)
    for (int l = t; l < Lv - 1; ++l) {
      const LevelDesc L = level_of(D, l);
      int cur = first_dst;
      if (nu >= 2) {
        tail_rows(L.n, [&](long long j) { body_jacobi_first2(D, L, l, j, first_dst, 0); });
        for (int s = 2; s < nu; ++s) {
          const int src = cur, dst = other_x(cur);
          tail_rows(L.n, [&](long long j) { body_jacobi(D, L, l, j, 0, src, dst, 0); });
          cur = dst;
        }
      } else {
        tail_rows(L.n, [&](long long j) { body_jacobi(D, L, l, j, 1, LB_X, first_dst, 0); });
      }
      if (cur == LB_X) cur_is_x |= 1u << l;
      const LevelDesc C = level_of(D, l + 1);
      const int xs = cur;
      for (long long g = threadIdx.x; 2 * g < C.n; g += kTailBlock)
        body_restrict(D, L, C, l, 2 * g, xs, 0);
      __syncthreads();
    }
    tail_coarse_solve(D, level_of(D, Lv - 1), bs);
    for (int l = Lv - 2; l >= t; --l) {
      const LevelDesc L = level_of(D, l);
      const LevelDesc C = level_of(D, l + 1);
      int cur = ((cur_is_x >> l) & 1u) ? LB_X : LB_T;
      {
        const int src = cur, dst = other_x(cur);
        tail_rows(L.n, [&](long long j) { body_jacobi_prolong(D, L, C, l, j, src, dst, 0); });
        cur = dst;
      }
      for (int s = 1; s < nu; ++s) {
        const int src = cur, dst = other_x(cur);
        tail_rows(L.n, [&](long long j) { body_jacobi(D, L, l, j, 0, src, dst, 0); });
        cur = dst;
      }
    }
  } else {
    const int m = sld(D.cheb_degree);
    for (int l = t; l < Lv - 1; ++l) {
      const LevelDesc L = level_of(D, l);
      const LevelDesc C = level_of(D, l + 1);
      for (int a = 0; a < nu; ++a) {
        int dcur = LB_T;
        int k0 = 0;
        if (a == 0) {
          float c_dd, c_dr;
          cheb_coefs(D, 0, c_dd, c_dr);
          const int last = (m == 1);
          tail_rows(L.n, [&](long long j) { body_cheb_first(D, L, l, j, last, LB_T, c_dd, c_dr); });
          k0 = 1;
        } else {
          tail_rows(L.n, [&](long long j) { body_cheb_start(D, L, l, j, 0, LB_T); });
        }
        for (int k = k0; k < m; ++k) {
          const int last = (k == m - 1);
          const int upd = !last || (a == nu - 1);
          const int dsel = dcur, dn = other_d(dcur);
          float c_dd, c_dr;
          cheb_coefs(D, k, c_dd, c_dr);
          tail_rows(L.n, [&](long long j) {
            body_cheb_step(D, L, C, l, j, 0, upd, last, dsel, dn, 0, 0, c_dd, c_dr);
          });
          dcur = dn;
        }
      }
      for (long long g = threadIdx.x; 2 * g < C.n; g += kTailBlock)
        body_restrict(D, L, C, l, 2 * g, LB_X, 1);
      __syncthreads();
    }
    tail_coarse_solve(D, level_of(D, Lv - 1), bs);
    for (int l = Lv - 2; l >= t; --l) {
      const LevelDesc L = level_of(D, l);
      const LevelDesc C = level_of(D, l + 1);
      for (int a = 0; a < nu; ++a) {
        if (a == 0)
          tail_rows(L.n, [&](long long j) { body_cheb_start_prolong(D, L, C, l, j, LB_T); });
        else
          tail_rows(L.n, [&](long long j) { body_cheb_start(D, L, l, j, 0, LB_T); });
        int dcur = LB_T;
        for (int k = 0; k < m; ++k) {
          const int last = (k == m - 1);
          const int dsel = dcur, dn = other_d(dcur);
          const int addp = (a == 0 && k == 0);
          float c_dd, c_dr;
          cheb_coefs(D, k, c_dd, c_dr);
          tail_rows(L.n, [&](long long j) {
            body_cheb_step(D, L, C, l, j, 0, !last, last, dsel, dn, 0, addp, c_dd, c_dr);
          });
          dcur = dn;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// launchers (n_l: voxels on level l; the level's nx must be a multiple of 4)
// ------------------------------------------------------------------------------------
static inline unsigned blocks4(long long n) {
  return (unsigned)((n / 4 + kBlock - 1) / kBlock);
}

#define LAUNCH4(kern, gx, gy, ...) \
  hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kBlock), 0, st, __VA_ARGS__)

int launch_jacobi4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int first,
                   int src, int dst, int want_dot) {
  const unsigned g = blocks4(n_l);
  LAUNCH4(k_jacobi4, g, B, d, l, first, src, dst, want_dot);
  return (int)g;
}
int launch_jacobi_first2_4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int dst,
                           int want_dot) {
  const unsigned g = blocks4(n_l);
  LAUNCH4(k_jacobi_first2_4, g, B, d, l, dst, want_dot);
  return (int)g;
}
int launch_jacobi_prolong4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int src,
                           int dst, int want_dot) {
  const unsigned g = blocks4(n_l);
  LAUNCH4(k_jacobi_prolong4, g, B, d, l, src, dst, want_dot);
  return (int)g;
}
void launch_cheb_first4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int last,
                        int dn_sel) {
  LAUNCH4(k_cheb_first4, blocks4(n_l), B, d, l, last, dn_sel);
}
void launch_cheb_start_prolong4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l,
                                int d_sel) {
  LAUNCH4(k_cheb_start_prolong4, blocks4(n_l), B, d, l, d_sel);
}
void launch_cheb_start4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int zero_x,
                        int d_sel) {
  LAUNCH4(k_cheb_start4, blocks4(n_l), B, d, l, zero_x, d_sel);
}
int launch_cheb_step4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int set_x,
                      int update_r, int last, int d_sel, int dn_sel, int step, int want_dot,
                      int add_prolong) {
  const unsigned g = blocks4(n_l);
  LAUNCH4(k_cheb_step4, g, B, d, l, set_x, update_r, last, d_sel, dn_sel, step, want_dot,
          add_prolong);
  return (int)g;
}
void launch_restrict4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse,
                      int x_sel, int use_r) {
  const unsigned g = (unsigned)((n_coarse / 2 + kBlock - 1) / kBlock);
  LAUNCH4(k_restrict4, g, B, d, l, x_sel, use_r);
}

void launch_vcycle_tail(hipStream_t st, InstDesc *const *d, int B, int t) {
  hipLaunchKernelGGL(k_vcycle_tail, dim3(1, B), dim3(kTailBlock), 0, st, d, t);
}

}  // namespace plsqr
