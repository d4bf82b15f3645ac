// Device helpers shared by the HIP kernel files (descriptor access, block reductions,
// diffusivity/penalty closed forms, the grid stencil and the product epilogues).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "plsqr_internal.hpp"

namespace plsqr {

// ------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ const InstDesc &inst(InstDesc *const *descs) {
  return *descs[blockIdx.y];
}

// Tile handled by this block. Workgroups are dealt to the 8 XCDs round-robin; when the grid
// splits evenly, consecutive tiles are given to blocks on the same XCD, so data that
// neighbouring tiles share (stencil and blur halos) is found in that XCD's L2.
__device__ __forceinline__ long long xcd_tile() {
  const unsigned b = blockIdx.x, nb = gridDim.x;
  if (nb % 8u != 0u) return b;
  return (long long)(b % 8u) * (nb / 8u) + b / 8u;
}

// This block's instance (index into the descriptor array; -1: a block between the ranges of a
// ragged launch), its block index within the instance and the instance's block count.
struct Blk {
  int i, bx, gx;
};
__device__ __forceinline__ Blk locate(const Rag &rg) {
  if (rg.n == 0) return Blk{(int)blockIdx.y, (int)blockIdx.x, (int)gridDim.x};
  const int b = blockIdx.x;
  Blk k{-1, 0, 0};
  for (int e = 0; e < rg.n; ++e)
    if (b >= rg.first[e] && b < rg.first[e] + rg.count[e]) k = Blk{rg.inst[e], b - rg.first[e], rg.count[e]};
  return k;
}
// xcd_tile for a block of a possibly ragged launch (an instance's range starts at a multiple of
// 8, so its block bx sits on XCD bx % 8 as in a uniform launch).
__device__ __forceinline__ long long xcd_tile_of(const Blk &k) {
  const unsigned b = k.bx, nb = k.gx;
  if (nb % 8u != 0u) return b;
  return (long long)(b % 8u) * (nb / 8u) + b / 8u;
}

// Uniform read of a descriptor field through the scalar cache. Descriptors are written by the
// host before the kernels that read them and never by a kernel, so they can be read as
// constant memory: one scalar load into SGPRs instead of a vector load per lane (which would
// sit on every kernel's critical path ahead of its first data load). Only descriptor fields
// go through here, never data that kernels write.
template <class T>
__device__ __forceinline__ T sld(const T &field) {
  return *(const __attribute__((address_space(4))) T *)(&field);
}

// Level l's descriptor, field by field through the scalar cache.
__device__ __forceinline__ LevelDesc level_of(const InstDesc &D, int l) {
  const LevelDesc &g = D.lv[l];
  LevelDesc L;
  L.nx = sld(g.nx);
  L.ny = sld(g.ny);
  L.nz = sld(g.nz);
  L.pad = 0;
  L.n = sld(g.n);
  L.x = sld(g.x);
  L.b = sld(g.b);
  L.r = sld(g.r);
  L.t = sld(g.t);
  L.s = sld(g.s);
  L.wx = sld(g.wx);
  L.wy = sld(g.wy);
  L.wz = sld(g.wz);
  L.dinv = sld(g.dinv);
  L.eps = sld(g.eps);
  return L;
}

// Adaptive stops (only for problems that request them): work that can no longer change the
// result is skipped. stopped_inner: MLSQR has ended in this outer step (S4, breakdown) or the
// outer loop has ended; stopped_outer: the outer loop has ended. The flags live in the scalar
// block, which kernels write, so they are read with ordinary loads.
__device__ __forceinline__ bool stopped_inner(const InstDesc &D) {
  return sld(D.stop_flags) != 0 && sld(D.sc)[SC_STOP] != 0.0;
}
__device__ __forceinline__ bool stopped_outer(const InstDesc &D) {
  return sld(D.stop_flags) != 0 && sld(D.sc)[SC_HALT] != 0.0;
}
// Strips the mask bits from a product's epilogue code; true if this instance skips the launch.
__device__ __forceinline__ bool product_masked(const InstDesc &D, int &epi) {
  const int m = epi & (EPI_MASK_INNER | EPI_MASK_OUTER);
  epi &= ~(EPI_MASK_INNER | EPI_MASK_OUTER);
  if (m == EPI_MASK_INNER) return stopped_inner(D);
  if (m == EPI_MASK_OUTER) return stopped_outer(D);
  return false;
}

__device__ __forceinline__ float *vec_of(const InstDesc &D, int sel) {
  switch (sel) {
    case V_F: return sld(D.f);
    case V_U: return sld(D.u);
    case V_P: return sld(D.p);
    case V_V: return sld(D.v);
    case V_W: return sld(D.w);
    case V_TMP1: return sld(D.tmp1);
    case V_TMP2: return sld(D.tmp2);
    default: return const_cast<float *>(sld(D.g));
  }
}

__device__ __forceinline__ float *lvbuf(const LevelDesc &L, int sel) {
  switch (sel) {
    case LB_X: return L.x;
    case LB_B: return L.b;
    case LB_R: return L.r;
    case LB_T: return L.t;
    default: return L.s;
  }
}

// Sum of v over the block (valid in thread 0). blockDim.x must be kBlock.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) r += red[i];
  return r;
}

__device__ __forceinline__ float block_sum_f(float v) {
  __shared__ float redf[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) redf[wid] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) r += redf[i];
  return r;
}

// kappa(t) = r'(t)/t in closed form (eq. (1.12)-(1.13) with r from (1.3)-(1.5)).
__device__ __forceinline__ float kappa_of(int reg, float t, float T) {
  switch (reg) {
    case PLSQR_REG_STV: return 1.0f / sqrtf(T * T + t * t);
    case PLSQR_REG_PM_LOG: return 1.0f / (1.0f + (t * t) / (T * T));
    case PLSQR_REG_PM_EXP: return expf(-(t * t) / (T * T));
    default: return 1.0f;
  }
}

// r(t), eq. (1.3)-(1.5), in FP64.
__device__ __forceinline__ double penalty_of(int reg, double t, double T) {
  switch (reg) {
    case PLSQR_REG_STV: return T * sqrt(1.0 + (t / T) * (t / T));
    case PLSQR_REG_PM_LOG: return 0.5 * T * T * log1p((t / T) * (t / T));
    case PLSQR_REG_PM_EXP: return 0.5 * T * T * (1.0 - exp(-(t * t) / (T * T)));
    default: return 0.5 * t * t;
  }
}

struct Coord { int x, y, z; };
// Grid coordinates of linear index j (x fastest). Grids hold < 2^31 cells (checked at
// submission), so 32-bit unsigned arithmetic suffices (64-bit division is emulated).
__device__ __forceinline__ Coord coord_of(long long j, int nx, int ny) {
  const unsigned u = (unsigned)j, ux = (unsigned)nx, uy = (unsigned)ny;
  const unsigned q = u / ux;
  Coord c;
  c.x = (int)(u - q * ux);
  c.y = (int)(q % uy);
  c.z = (int)(q / uy);
  return c;
}

// (A_l x)_j on level l: eps_l x_j + sum over the faces of cell j of w (x_j - x_nb).
// Level 0 face weight to the +a neighbour is kappa_j; coarser levels store them.
__device__ __forceinline__ float stencil(const InstDesc &D, int l, const float *__restrict__ x,
                                         long long j, Coord c) {
  const LevelDesc L = level_of(D, l);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const long long sx = 1, sy = nx, sz = (long long)nx * ny;
  const float xj = x[j];
  float acc = (float)L.eps * xj;
  if (l == 0) {
    const float *__restrict__ k = sld(D.kappa);
    const float kj = k[j];
    if (c.x + 1 < nx) acc += kj * (xj - x[j + sx]);
    if (c.x > 0) acc += k[j - sx] * (xj - x[j - sx]);
    if (c.y + 1 < ny) acc += kj * (xj - x[j + sy]);
    if (c.y > 0) acc += k[j - sy] * (xj - x[j - sy]);
    if (c.z + 1 < nz) acc += kj * (xj - x[j + sz]);
    if (c.z > 0) acc += k[j - sz] * (xj - x[j - sz]);
  } else {
    if (c.x + 1 < nx) acc += L.wx[j] * (xj - x[j + sx]);
    if (c.x > 0) acc += L.wx[j - sx] * (xj - x[j - sx]);
    if (c.y + 1 < ny) acc += L.wy[j] * (xj - x[j + sy]);
    if (c.y > 0) acc += L.wy[j - sy] * (xj - x[j - sy]);
    if (nz > 1) {
      if (c.z + 1 < nz) acc += L.wz[j] * (xj - x[j + sz]);
      if (c.z > 0) acc += L.wz[j - sz] * (xj - x[j - sz]);
    }
  }
  return acc;
}

// (A_l x)_j together with 1/diag(A_l)_j. On level 0 the diagonal eps + sum of the face
// weights is assembled from the kappa values the stencil loads anyway (same order of
// additions as the stored level-0 diagonal), so the level-0 smoother kernels need not read
// a diagonal array; coarser levels read their stored 1/diag.
__device__ __forceinline__ float stencil_dinv(const InstDesc &D, int l, const float *__restrict__ x,
                                              long long j, Coord c, float &dinv_j) {
  if (l != 0) {
    dinv_j = sld(D.lv[l].dinv)[j];
    return stencil(D, l, x, j, c);
  }
  const LevelDesc L = level_of(D, 0);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const long long sy = nx, sz = (long long)nx * ny;
  const float *__restrict__ k = sld(D.kappa);
  const float xj = x[j];
  const float kj = k[j];
  float acc = (float)L.eps * xj;
  float dg = (float)L.eps;
  if (c.x + 1 < nx) { acc += kj * (xj - x[j + 1]); dg += kj; }
  if (c.x > 0) { const float kk = k[j - 1]; acc += kk * (xj - x[j - 1]); dg += kk; }
  if (c.y + 1 < ny) { acc += kj * (xj - x[j + sy]); dg += kj; }
  if (c.y > 0) { const float kk = k[j - sy]; acc += kk * (xj - x[j - sy]); dg += kk; }
  if (c.z + 1 < nz) { acc += kj * (xj - x[j + sz]); dg += kj; }
  if (c.z > 0) { const float kk = k[j - sz]; acc += kk * (xj - x[j - sz]); dg += kk; }
  dinv_j = 1.0f / dg;
  return acc;
}

// (A_l x)_j where the values of x come from a functor X(index): used when the iterate is
// formed on the fly (first Jacobi sweep from zero, prolongated correction).
template <class XF>
__device__ __forceinline__ float stencil_f(const InstDesc &D, int l, long long j, Coord c,
                                           XF X) {
  const LevelDesc L = level_of(D, l);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const long long sy = nx, sz = (long long)nx * ny;
  const float xj = X(j, c);
  float acc = (float)L.eps * xj;
  auto nb = [&](int dx, int dy, int dz) {
    Coord q = c;
    q.x += dx;
    q.y += dy;
    q.z += dz;
    return q;
  };
  if (l == 0) {
    const float *__restrict__ k = sld(D.kappa);
    const float kj = k[j];
    if (c.x + 1 < nx) acc += kj * (xj - X(j + 1, nb(1, 0, 0)));
    if (c.x > 0) acc += k[j - 1] * (xj - X(j - 1, nb(-1, 0, 0)));
    if (c.y + 1 < ny) acc += kj * (xj - X(j + sy, nb(0, 1, 0)));
    if (c.y > 0) acc += k[j - sy] * (xj - X(j - sy, nb(0, -1, 0)));
    if (c.z + 1 < nz) acc += kj * (xj - X(j + sz, nb(0, 0, 1)));
    if (c.z > 0) acc += k[j - sz] * (xj - X(j - sz, nb(0, 0, -1)));
  } else {
    if (c.x + 1 < nx) acc += L.wx[j] * (xj - X(j + 1, nb(1, 0, 0)));
    if (c.x > 0) acc += L.wx[j - 1] * (xj - X(j - 1, nb(-1, 0, 0)));
    if (c.y + 1 < ny) acc += L.wy[j] * (xj - X(j + sy, nb(0, 1, 0)));
    if (c.y > 0) acc += L.wy[j - sy] * (xj - X(j - sy, nb(0, -1, 0)));
    if (nz > 1) {
      if (c.z + 1 < nz) acc += L.wz[j] * (xj - X(j + sz, nb(0, 0, 1)));
      if (c.z > 0) acc += L.wz[j - sz] * (xj - X(j - sz, nb(0, 0, -1)));
    }
  }
  return acc;
}

// ---- 4-wide stencils (x-vectorised: thread owns voxels j..j+3, x0 = c.x % 4 == 0) -------
struct V4 {
  float v[4];
};
__device__ __forceinline__ V4 ld4(const float *p) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  V4 r;
  r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  return r;
}
__device__ __forceinline__ void st4(float *p, const V4 &a) {
  *reinterpret_cast<float4 *>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
}

// (A_l x) and 1/diag(A_l) for the 4 voxels j..j+3 of one x-row (c.x % 4 == 0, nx % 4 == 0).
// xc is the iterate at j..j+3; X4(idx, coord) returns it at idx..idx+3 (coord of idx) for the
// y and z neighbours, X1(idx, coord) one value (the two x-neighbours). Face weights and
// diagonals are accumulated in the same order as the one-voxel stencils above, so both give
// the same values.
// L is level l's view (level_of(D, l)).
template <class F4, class F1>
__device__ __forceinline__ V4 stencil4(const InstDesc &D, const LevelDesc &L, int l, long long j,
                                       Coord c, const V4 &xc, F4 X4, F1 X1, V4 &dinv) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const long long sy = nx, sz = (long long)nx * ny;
  Coord cl = c, cr = c;
  cl.x -= 1;
  cr.x += 4;
  const float xl = (c.x > 0) ? X1(j - 1, cl) : 0.f;
  const float xr = (c.x + 4 < nx) ? X1(j + 4, cr) : 0.f;
  Coord cyp = c, cym = c, czp = c, czm = c;
  cyp.y += 1; cym.y -= 1; czp.z += 1; czm.z -= 1;
  V4 yp = {}, ym = {}, zp = {}, zm = {};
  const bool hyp = c.y + 1 < ny, hym = c.y > 0, hzp = c.z + 1 < nz, hzm = c.z > 0;
  if (hyp) yp = X4(j + sy, cyp);
  if (hym) ym = X4(j - sy, cym);
  if (hzp) zp = X4(j + sz, czp);
  if (hzm) zm = X4(j - sz, czm);
  // face weights: wxp[e] (to e+1), wxm0 (from x0-1), wy/wym, wz/wzm
  V4 wxp, wyp, wym = {}, wzp = {}, wzm = {};
  float wxm0;
  if (l == 0) {
    const float *kappa = sld(D.kappa);
    const V4 k = ld4(kappa + j);
    wxp = k; wyp = k; wzp = k;
    wxm0 = (c.x > 0) ? kappa[j - 1] : 0.f;
    if (hym) wym = ld4(kappa + j - sy);
    if (hzm) wzm = ld4(kappa + j - sz);
  } else {
    wxp = ld4(L.wx + j);
    wyp = ld4(L.wy + j);
    wxm0 = (c.x > 0) ? L.wx[j - 1] : 0.f;
    if (hym) wym = ld4(L.wy + j - sy);
    if (nz > 1) {
      wzp = ld4(L.wz + j);
      if (hzm) wzm = ld4(L.wz + j - sz);
    }
  }
  V4 out;
  const float eps = (float)L.eps;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float xj = xc.v[e];
    float acc = eps * xj;
    float dg = eps;
    const bool hxp = c.x + e + 1 < nx;
    const bool hxm = c.x + e > 0;
    const float xnext = (e < 3) ? xc.v[e < 3 ? e + 1 : 3] : xr;
    const float xprev = (e > 0) ? xc.v[e > 0 ? e - 1 : 0] : xl;
    const float wm = (e > 0) ? wxp.v[e > 0 ? e - 1 : 0] : wxm0;
    if (hxp) { acc += wxp.v[e] * (xj - xnext); dg += wxp.v[e]; }
    if (hxm) { acc += wm * (xj - xprev); dg += wm; }
    if (hyp) { acc += wyp.v[e] * (xj - yp.v[e]); dg += wyp.v[e]; }
    if (hym) { acc += wym.v[e] * (xj - ym.v[e]); dg += wym.v[e]; }
    if (nz > 1 || l == 0) {
      if (hzp) { acc += wzp.v[e] * (xj - zp.v[e]); dg += wzp.v[e]; }
      if (hzm) { acc += wzm.v[e] * (xj - zm.v[e]); dg += wzm.v[e]; }
    }
    out.v[e] = acc;
    dinv.v[e] = 1.0f / dg;
  }
  if (l != 0) dinv = ld4(L.dinv + j);
  return out;
}

// Index of the coarse parent of fine cell (c) on level l (2:1 in x, y and, in 3D, z).
__device__ __forceinline__ long long parent_of(const LevelDesc &F, const LevelDesc &Cl, Coord c) {
  const int cz = (F.nz > 1) ? 2 : 1;
  return (c.x >> 1) + (long long)Cl.nx * ((c.y >> 1) + (long long)Cl.ny * (c.z / cz));
}

__device__ __forceinline__ void epilogue(const InstDesc &D, int epi, long long j, float y,
                                         float *out, double &dot) {
  const double *sc = sld(D.sc);
  switch (epi) {
    case EPI_FWD: {
      float *u = sld(D.u);
      const float c1 = (float)sc[SC_SV], c2 = (float)(sc[SC_ALPHA] * sc[SC_SU]);
      const float un = c1 * y - c2 * u[j];
      u[j] = un;
      dot = (double)un * (double)un;
      break;
    }
    case EPI_ADJ: {
      float *p = sld(D.p);
      const float c1 = (float)sc[SC_SU], c2 = (float)(sc[SC_BETA] * sc[SC_SV]);
      p[j] = c1 * y - c2 * p[j];
      break;
    }
    case EPI_ADJ_INIT: sld(D.p)[j] = (float)sc[SC_SU] * y; break;
    case EPI_RESID: {
      const double e = (double)sld(D.g)[j] - (double)y;
      dot = e * e;
      break;
    }
    default: out[j] = y; break;
  }
}

}  // namespace plsqr
