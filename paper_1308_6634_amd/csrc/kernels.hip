// HIP kernels (gfx950) of the priorconditioned lagged-diffusivity solver.
//
// Every kernel is batched: blockIdx.y selects an instance through a device array of
// InstDesc pointers, blockIdx.x tiles that instance's grid. Blocks past an instance's
// extent still take part in block reductions (they contribute 0), so every reduction
// writes exactly gridDim.x partials per instance, which one finaliser block then sums
// in a fixed order (deterministic FP64 reductions).
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.hpp"
#include "finalize.hpp"
#include "kernels.hpp"

namespace plsqr {

// ------------------------------------------------------------------------------------
// Lagged diffusivity: |grad f|, c_f = r'(t)/t of eqs. (1.12)-(1.13) and R(f) (section 4.1)
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_diffusivity(InstDesc *const *descs, int write_kappa) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double r = 0.0;
  if (j < sld(D.n)) {
    const int nx = sld(D.nx), ny = sld(D.ny), nz = sld(D.nz);
    const Coord c = coord_of(j, nx, ny);
    const float *__restrict__ f = sld(D.f);
    const float fj = f[j];
    const float gx = (c.x + 1 < nx) ? f[j + 1] - fj : 0.f;
    const float gy = (c.y + 1 < ny) ? f[j + nx] - fj : 0.f;
    const float gz = (c.z + 1 < nz) ? f[j + (long long)nx * ny] - fj : 0.f;
    const float t = sqrtf(gx * gx + gy * gy + gz * gz);
    if (write_kappa) sld(D.kappa)[j] = kappa_of(sld(D.reg), t, sld(D.T));
    r = penalty_of(sld(D.reg), (double)t, (double)sld(D.T));
  }
  r = block_sum(r);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = r;
}

// ------------------------------------------------------------------------------------
// Multigrid hierarchy (Galerkin face sums), diagonals, coarsest Cholesky (section 4.2)
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_level0_dinv(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= sld(D.n)) return;
  const int nx = sld(D.nx), ny = sld(D.ny), nz = sld(D.nz);
  const Coord c = coord_of(j, nx, ny);
  const float *__restrict__ k = sld(D.kappa);
  const long long sy = nx, sz = (long long)nx * ny;
  const float kj = k[j];
  float d = (float)sld(D.lv[0].eps);
  if (c.x + 1 < nx) d += kj;
  if (c.x > 0) d += k[j - 1];
  if (c.y + 1 < ny) d += kj;
  if (c.y > 0) d += k[j - sy];
  if (c.z + 1 < nz) d += kj;
  if (c.z > 0) d += k[j - sz];
  sld(D.lv[0].dinv)[j] = 1.0f / d;
}

// Face weight of the fine level l from cell j to its +a neighbour (0 outside the grid).
__device__ __forceinline__ float face_w(const InstDesc &D, int l, int a, long long j, Coord c) {
  const LevelDesc L = level_of(D, l);
  if (l == 0) {
    const bool in = (a == 0) ? (c.x + 1 < L.nx) : (a == 1) ? (c.y + 1 < L.ny) : (c.z + 1 < L.nz);
    return in ? sld(D.kappa)[j] : 0.f;
  }
  return (a == 0) ? L.wx[j] : (a == 1) ? L.wy[j] : L.wz[j];
}

// Galerkin coarsening l -> l+1 with piecewise-constant P: the weight of coarse face
// (J, J+e_a) is the sum of the fine face weights crossing it.
__global__ void __launch_bounds__(kBlock) k_coarsen(InstDesc *const *descs, int l) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const LevelDesc F = level_of(D, l);
  const LevelDesc Cl = level_of(D, l + 1);
  const long long J = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (J >= Cl.n) return;
  const Coord cc = coord_of(J, Cl.nx, Cl.ny);
  const int cz = (F.nz > 1) ? 2 : 1;
  // a coarse level with one z-plane (a 3D grid coarsened to nz = 1) has no z faces and no wz
  // array; its cells still have 2 z children when the fine level has two planes
  const int naxes = (Cl.nz > 1) ? 3 : 2;
  for (int a = 0; a < naxes; ++a) {
    float s = 0.f;
    // children of J with local coordinate 1 along a (their +a face leaves J)
    for (int dz = 0; dz < cz; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int lx = dx, ly = dy, lz = dz;
          const int loc = (a == 0) ? lx : (a == 1) ? ly : lz;
          if (loc != 1) continue;
          Coord fc;
          fc.x = 2 * cc.x + dx;
          fc.y = 2 * cc.y + dy;
          fc.z = cz * cc.z + dz;
          const long long j = fc.x + (long long)F.nx * (fc.y + (long long)F.ny * fc.z);
          s += face_w(D, l, a, j, fc);
        }
    float *dst = (a == 0) ? Cl.wx : (a == 1) ? Cl.wy : Cl.wz;
    dst[J] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_level_dinv(InstDesc *const *descs, int l) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= L.n) return;
  const Coord c = coord_of(j, L.nx, L.ny);
  const long long sy = L.nx, sz = (long long)L.nx * L.ny;
  float d = (float)L.eps;
  d += L.wx[j] + (c.x > 0 ? L.wx[j - 1] : 0.f);
  d += L.wy[j] + (c.y > 0 ? L.wy[j - sy] : 0.f);
  if (L.nz > 1) d += L.wz[j] + (c.z > 0 ? L.wz[j - sz] : 0.f);
  L.dinv[j] = 1.0f / d;
}

// Coarsest grids of up to kCoarseLds cells are inverted in LDS (coarse_gj_inverse, kCoarseLdsRows
// rows per thread), larger ones in the instance's FP64 workspace (coarse_factor_body).
constexpr int kCoarseLds = 64;
constexpr int kCoarseLdsRows = kCoarseLds / (kBlock / 64);

// Assemble the coarsest operator densely in FP64 into at(i, j) (all n x n entries written).
template <class At>
__device__ __forceinline__ void coarse_assemble(const InstDesc &D, const LevelDesc &L, int l, int n,
                                                At at) {
  // (n <= 512: 32-bit indices; wave w takes rows w, w + 4, .., lane c columns c, c + 64, ..)
  for (int i = (int)(threadIdx.x >> 6); i < n; i += kBlock / 64)
    for (int j = (int)(threadIdx.x & 63); j < n; j += 64) at(i, j) = 0.0;
  __syncthreads();
  for (int J = threadIdx.x; J < n; J += kBlock) {
    const Coord c = coord_of(J, L.nx, L.ny);
    const int strides[3] = {1, L.nx, L.nx * L.ny};
    const int ext[3] = {L.nx, L.ny, L.nz};
    const int pos[3] = {c.x, c.y, c.z};
    double diag = L.eps;
    for (int a = 0; a < 3; ++a) {
      if (ext[a] == 1) continue;
      if (pos[a] + 1 < ext[a]) {
        const double w = face_w(D, l, a, J, c);
        diag += w;
        at(J, J + strides[a]) = -w;
      }
      if (pos[a] > 0) {
        Coord cm = c;
        if (a == 0) cm.x -= 1; else if (a == 1) cm.y -= 1; else cm.z -= 1;
        const double w = face_w(D, l, a, J - strides[a], cm);
        diag += w;
        at(J, J - strides[a]) = -w;
      }
    }
    at(J, J) = diag;
  }
}

// The inverse of the assembled coarsest operator (n <= 64, in LDS) by in-place Gauss-Jordan
// elimination without pivoting: step k scales row k by 1 / a_kk and eliminates column k from
// every other row. For a symmetric positive definite matrix the pivots are those of its
// Cholesky factorisation (the Schur complements), so a non-positive one flags the matrix as not
// SPD (and is replaced by 1, as the factorisation path does). Each step reads row and column k
// from snapshots (rowk, colk: n doubles of LDS each), so every entry is updated by the one
// thread that owns it, from values no other thread writes during the step: two barriers a step.
template <class At>
__device__ __forceinline__ void coarse_gj_inverse(int n, At at, double *rowk, double *colk,
                                                  double *Ainv, int &bad) {
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);   // lane: column j
  constexpr int kWaves = kBlock / 64;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int i = threadIdx.x; i < n; i += kBlock) {
      colk[i] = at(i, k);
      rowk[i] = at(k, i);
    }
    __syncthreads();
    double piv = colk[k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) bad = 1;
      piv = 1.0;
    }
    const double rp = 1.0 / piv;
    if (lane < n) {
      const int j = lane;
      const double rj = ((j == k) ? 1.0 : rowk[j]) * rp;   // row k after its scaling
      double aij[kCoarseLdsRows];
#pragma unroll
      for (int r = 0; r < kCoarseLdsRows; ++r) {
        const int i = min(w + kWaves * r, n - 1);   // clamped: read, never written
        aij[r] = at(i, j);
      }
#pragma unroll
      for (int r = 0; r < kCoarseLdsRows; ++r) {
        const int i = w + kWaves * r;
        if (i >= n) continue;
        if (i == k) at(i, j) = rj;
        else at(i, j) = ((j == k) ? 0.0 : aij[r]) - colk[i] * rj;
      }
    }
    __syncthreads();
  }
  for (int i = w; i < n; i += kWaves)
    if (lane < n) Ainv[i * n + lane] = at(i, lane);
}

// The global-memory path (64 < n <= 512): factor the assembled operator (lower Cholesky,
// right-looking, in place) and form its explicit inverse A^{-1} = L^{-T} L^{-1}, so that each
// V-cycle's coarsest solve is one parallel matrix-vector product. at(i, j) is the working
// matrix: its lower triangle holds L, and L^{-1} (formed column by column, one thread per
// column) is kept transposed in the strict upper triangle with its diagonal in dv. A^{-1} goes
// to Ainv.
template <class At, class Dv>
__device__ __forceinline__ void coarse_factor_body(const InstDesc &D, const LevelDesc &L, int l,
                                                   int n, At at, Dv dv, double *Ainv, int &bad) {
  coarse_assemble(D, L, l, n, at);
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double d = at(k, k);
      if (!(d > 0.0)) { bad = 1; d = 1.0; }
      at(k, k) = sqrt(d);
    }
    __syncthreads();
    const double piv = at(k, k);
    for (int i = k + 1 + threadIdx.x; i < n; i += kBlock) at(i, k) /= piv;
    __syncthreads();
    // the trailing lower triangle: lane c takes the columns jj = k + 1 + c, k + 1 + c + 64, ..,
    // wave w the rows i = k + 1 + w, k + 1 + w + 4, .. (i >= jj), eight rows at a time with all
    // their reads issued before their updates (a row at a time waits on three dependent LDS
    // accesses)
    constexpr int kRows = 8, kWaves = kBlock / 64;
    for (int jj = k + 1 + (int)(threadIdx.x & 63); jj < n; jj += 64) {
      const double ajk = at(jj, k);
      for (int i0 = k + 1 + (int)(threadIdx.x >> 6); i0 < n; i0 += kRows * kWaves) {
        double lik[kRows], aij[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int i = min(i0 + kWaves * r, n - 1);   // clamped: read, never written
          lik[r] = at(i, k);
          aij[r] = at(i, jj);
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int i = i0 + kWaves * r;
          if (i < n && jj <= i) at(i, jj) = aij[r] - lik[r] * ajk;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) {
    sld(D.sc)[SC_STATUS] = (double)PLSQR_E_NOT_SPD;
    sld(D.sc)[SC_STOP] = 1.0;
  }
  // L^{-1}[k][j] (k >= j) is dv[j] on the diagonal and at(j, k) below it. The sums below run
  // in four interleaved partial sums (k = k0 + 4 m + e), so that four of their loads are in
  // flight at once instead of one dependent load per term.
  auto li = [&](int k, int j) -> double { return k == j ? dv[j] : at(j, k); };
  for (int j = threadIdx.x; j < n; j += kBlock) {
    for (int i = j; i < n; ++i) {
      double s4[4] = {(i == j) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
      int k = j;
      for (; k + 3 < i; k += 4)
#pragma unroll
        for (int e = 0; e < 4; ++e) s4[e] -= at(i, k + e) * li(k + e, j);
      for (; k < i; ++k) s4[0] -= at(i, k) * li(k, j);
      const double v = ((s4[0] + s4[1]) + (s4[2] + s4[3])) / at(i, i);
      if (i == j) dv[j] = v; else at(j, i) = v;
    }
  }
  __syncthreads();
  // A^{-1}[i][j] = sum_{k >= max(i,j)} L^{-1}[k][i] L^{-1}[k][j]
  for (int i = (int)(threadIdx.x >> 6); i < n; i += kBlock / 64) {
    for (int j = (int)(threadIdx.x & 63); j < n; j += 64) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int k = i > j ? i : j;
      for (; k + 3 < n; k += 4)
#pragma unroll
        for (int e = 0; e < 4; ++e) s4[e] += li(k + e, i) * li(k + e, j);
      for (; k < n; ++k) s4[0] += li(k, i) * li(k, j);
      Ainv[i * n + j] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
  }
}

// One block per instance: A^{-1} of the coarsest operator, in LDS (Gauss-Jordan) up to
// kCoarseLds cells, else in the instance's FP64 workspace (cfac: working matrix, L^{-1}
// diagonal, A^{-1}; Cholesky).
__global__ void __launch_bounds__(kBlock) k_coarse_factor(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const int l = sld(D.levels) - 1;
  const LevelDesc L = level_of(D, l);
  const int n = (int)L.n;
  double *__restrict__ W = sld(D.cfac);
  double *Ainv = W + (long long)n * n * 2;
  // rows n + 1 doubles apart: the lanes of a wave that read one column of consecutive rows hit
  // different banks (n doubles apart, a power of two, they would all hit the same bank)
  __shared__ double S[kCoarseLds * (kCoarseLds + 1)];
  __shared__ double srow[kCoarseLds], scol[kCoarseLds];
  __shared__ int bad;
  if (n <= kCoarseLds) {
    auto at = [&](int i, int j) -> double & { return S[i * (n + 1) + j]; };
    coarse_assemble(D, L, l, n, at);
    coarse_gj_inverse(n, at, srow, scol, Ainv, bad);
    if (threadIdx.x == 0 && bad) {
      sld(D.sc)[SC_STATUS] = (double)PLSQR_E_NOT_SPD;
      sld(D.sc)[SC_STOP] = 1.0;
    }
  } else {
    double *gdv = W + (long long)n * n;
    coarse_factor_body(D, L, l, n,
                       [&](int i, int j) -> double & { return W[(long long)i * n + j]; }, gdv,
                       Ainv, bad);
  }
}

// Coarsest solve: x = A_c^{-1} b with the FP64 inverse formed at setup (symmetric, so
// thread i reads column i: coalesced). One block per instance.
__global__ void __launch_bounds__(kBlock) k_coarse_solve(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, sld(D.levels) - 1);
  const int n = (int)L.n;
  const double *__restrict__ Ai = sld(D.cfac) + (long long)n * n * 2;
  __shared__ double bs[PLSQR_MAX_COARSE];
  for (int i = threadIdx.x; i < n; i += kBlock) bs[i] = (double)L.b[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += Ai[(long long)j * n + i] * bs[j];
    L.x[i] = (float)acc;
  }
}

// ------------------------------------------------------------------------------------
// V-cycle pieces (section 4.2)
// ------------------------------------------------------------------------------------
// Damped Jacobi sweep dst = src + omega D^{-1} (b - A src)  (first: src = 0).
// With want_dot, also the partial of sum_j dst_j b_j (alpha^2 on level 0).
__global__ void __launch_bounds__(kBlock) k_jacobi(InstDesc *const *descs, int l, int first,
                                                  int src_sel, int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < L.n) {
    const float *__restrict__ b = L.b;
    float *dst = lvbuf(L, dst_sel);
    float xn;
    if (first) {
      xn = sld(D.omega) * L.dinv[j] * b[j];
    } else {
      const float *__restrict__ src = lvbuf(L, src_sel);
      const Coord c = coord_of(j, L.nx, L.ny);
      float dv;
      const float ax = stencil_dinv(D, l, src, j, c, dv);
      xn = src[j] + sld(D.omega) * dv * (b[j] - ax);
    }
    dst[j] = xn;
    if (want_dot) dot = (double)xn * (double)b[j];
  }
  if (want_dot) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
  }
}

// First two damped Jacobi sweeps from x = 0 in one pass: x1 = omega D^{-1} b is formed on
// the fly (also at the neighbours), dst = x1 + omega D^{-1} (b - A x1).
__global__ void __launch_bounds__(kBlock) k_jacobi_first2(InstDesc *const *descs, int l,
                                                         int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < L.n) {
    const float *__restrict__ b = L.b;
    const float *__restrict__ dinv = L.dinv;
    const float om = sld(D.omega);
    const Coord c = coord_of(j, L.nx, L.ny);
    auto x1 = [&](long long q, Coord) { return om * dinv[q] * b[q]; };
    const float ax = stencil_f(D, l, j, c, x1);
    const float xn = x1(j, c) + om * dinv[j] * (b[j] - ax);
    lvbuf(L, dst_sel)[j] = xn;
    if (want_dot) dot = (double)xn * (double)b[j];
  }
  if (want_dot) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
  }
}

// Prolongation fused into the first post-smoothing Jacobi sweep: x' = x + P e (formed on
// the fly at the neighbours), dst = x' + omega D^{-1} (b - A x').
__global__ void __launch_bounds__(kBlock) k_jacobi_prolong(InstDesc *const *descs, int l,
                                                          int src_sel, int dst_sel, int want_dot) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const LevelDesc Cl = level_of(D, l + 1);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < L.n) {
    const float *__restrict__ x = lvbuf(L, src_sel);
    const float *__restrict__ e = Cl.x;
    const Coord c = coord_of(j, L.nx, L.ny);
    auto xp = [&](long long q, Coord cq) { return x[q] + e[parent_of(L, Cl, cq)]; };
    const float ax = stencil_f(D, l, j, c, xp);
    const float xn = xp(j, c) + sld(D.omega) * L.dinv[j] * (L.b[j] - ax);
    lvbuf(L, dst_sel)[j] = xn;
    if (want_dot) dot = (double)xn * (double)L.b[j];
  }
  if (want_dot) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
  }
}

// Chebyshev pre-smoothing start fused with its first step (x = 0): d0 = D^{-1} b / theta on
// the fly, x1 = d0, r1 = b - A d0, and (unless the polynomial has degree 1) d1 -> dn_sel.
__global__ void __launch_bounds__(kBlock) k_cheb_first(InstDesc *const *descs, int l, int last,
                                                      int dn_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= L.n) return;
  const double rho0 = 1.0 / sld(D.cheb_sigma);
  const double rho1 = 1.0 / (2.0 * sld(D.cheb_sigma) - rho0);
  const float c_dd = (float)(rho1 * rho0), c_dr = (float)(2.0 * rho1 / sld(D.cheb_delta));
  const float ith = (float)(1.0 / sld(D.cheb_theta));
  const float *__restrict__ b = L.b;
  const float *__restrict__ dinv = L.dinv;
  const Coord c = coord_of(j, L.nx, L.ny);
  auto d0 = [&](long long q, Coord) { return ith * dinv[q] * b[q]; };
  const float dj = d0(j, c);
  L.x[j] = dj;
  const float r = b[j] - stencil_f(D, l, j, c, d0);
  L.r[j] = r;
  if (!last) lvbuf(L, dn_sel)[j] = c_dd * dj + c_dr * dinv[j] * r;
}

// Chebyshev post-smoothing start fused with the prolongation: r = b - A x' with
// x' = x + P e formed on the fly (x itself is left alone: other blocks still read it; the
// first step adds P e pointwise), d = D^{-1} r / theta -> d_sel.
__global__ void __launch_bounds__(kBlock) k_cheb_start_prolong(InstDesc *const *descs, int l,
                                                              int d_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const LevelDesc Cl = level_of(D, l + 1);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= L.n) return;
  const float *__restrict__ x = L.x;
  const float *__restrict__ e = Cl.x;
  const Coord c = coord_of(j, L.nx, L.ny);
  auto xp = [&](long long q, Coord cq) { return x[q] + e[parent_of(L, Cl, cq)]; };
  const float r = L.b[j] - stencil_f(D, l, j, c, xp);
  L.r[j] = r;
  lvbuf(L, d_sel)[j] = (float)(1.0 / sld(D.cheb_theta)) * L.dinv[j] * r;
}

// Restriction of the residual with one thread per fine cell: the 2^d children of a coarse
// cell sit in consecutive lanes and are summed with shuffles.
// use_r: sum the stored residual r_l; otherwise form b - A_l x.
__global__ void __launch_bounds__(kBlock) k_restrict_fine(InstDesc *const *descs, int l, int x_sel,
                                                         int use_r) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc F = level_of(D, l);
  const LevelDesc Cl = level_of(D, l + 1);
  const int nchild = (F.nz > 1) ? 8 : 4;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long J = t / nchild;
  const int ch = (int)(t % nchild);
  float v = 0.f;
  if (J < Cl.n) {
    const Coord cc = coord_of(J, Cl.nx, Cl.ny);
    Coord fc;
    fc.x = 2 * cc.x + (ch & 1);
    fc.y = 2 * cc.y + ((ch >> 1) & 1);
    fc.z = (F.nz > 1) ? 2 * cc.z + (ch >> 2) : 0;
    const long long j = fc.x + (long long)F.nx * (fc.y + (long long)F.ny * fc.z);
    v = use_r ? F.r[j] : F.b[j] - stencil(D, l, lvbuf(F, x_sel), j, fc);
  }
  // sum over the nchild consecutive lanes (groups never straddle a wave: 64 % 8 == 0)
  for (int o = 1; o < nchild; o <<= 1) v += __shfl_xor(v, o, 64);
  if (J < Cl.n && ch == 0) Cl.b[J] = v;
}

// Chebyshev start: r = b - A x (or r = b when x = 0), d = D^{-1} r / theta -> d buffer.
__global__ void __launch_bounds__(kBlock) k_cheb_start(InstDesc *const *descs, int l, int zero_x,
                                                      int d_sel) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= L.n) return;
  float r = L.b[j];
  float dv;
  const Coord c = coord_of(j, L.nx, L.ny);
  if (!zero_x) {
    r -= stencil_dinv(D, l, L.x, j, c, dv);
  } else {
    dv = L.dinv[j];
  }
  L.r[j] = r;
  lvbuf(L, d_sel)[j] = (float)(1.0 / sld(D.cheb_theta)) * dv * r;
}

// One Chebyshev step: x += d (x = d when set_x); r -= A d (if update_r);
// d' = c_dd d + c_dr D^{-1} r (if !last). d is read from d_sel, d' written to dn_sel.
// With want_dot, partial of sum x_j b_j after the update.
__global__ void __launch_bounds__(kBlock) k_cheb_step(InstDesc *const *descs, int l, int set_x,
                                                     int update_r, int last, int d_sel, int dn_sel,
                                                     int step, int want_dot, int add_prolong) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const LevelDesc L = level_of(D, l);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  // rho_0 = 1/sigma, rho_{k+1} = 1/(2 sigma - rho_k); d' = rho_{k+1} rho_k d + 2 rho_{k+1}/delta D^{-1} r
  double rho = 1.0 / sld(D.cheb_sigma);
  for (int i = 0; i < step; ++i) rho = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  const double rho_next = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  const float c_dd = (float)(rho_next * rho), c_dr = (float)(2.0 * rho_next / sld(D.cheb_delta));
  double dot = 0.0;
  if (j < L.n) {
    const float *__restrict__ d = lvbuf(L, d_sel);
    const float dj = d[j];
    float xo = set_x ? 0.f : L.x[j];
    if (add_prolong) {      // pending coarse correction x += P e (pointwise)
      const LevelDesc Cl = level_of(D, l + 1);
      xo += Cl.x[parent_of(L, Cl, coord_of(j, L.nx, L.ny))];
    }
    const float xn = xo + dj;
    L.x[j] = xn;
    if (want_dot) dot = (double)xn * (double)L.b[j];
    if (update_r) {
      const Coord c = coord_of(j, L.nx, L.ny);
      float dv;
      const float r = L.r[j] - stencil_dinv(D, l, d, j, c, dv);
      L.r[j] = r;
      if (!last) lvbuf(L, dn_sel)[j] = c_dd * dj + c_dr * dv * r;
    }
  }
  if (want_dot) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
  }
}


// ------------------------------------------------------------------------------------
// Krylov recurrences: copies, reductions, rotations, updates (section 3.2, Algorithm 2)
// ------------------------------------------------------------------------------------
// Start of outer step k: reset the per-step Krylov flags.
__global__ void k_outer_begin(InstDesc *const *descs, int nblocks_unused) {
  const InstDesc &D = inst(descs);
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double *sc = sld(D.sc);
    if (sc[SC_HALT] != 0.0) return;   // the outer loop has stopped: this step changes nothing
    sc[SC_OUTER] += 1.0;
    sc[SC_STOP] = (sc[SC_STATUS] != 0.0) ? 1.0 : 0.0;
    sc[SC_DONE] = 0.0;
    sc[SC_SU] = 0.0;
    sc[SC_SV] = 0.0;
    sc[SC_ALPHA] = 0.0;
    sc[SC_BETA] = 0.0;
  }
  (void)nblocks_unused;
}

// Start of a request: zero f and the scalar block.
__global__ void __launch_bounds__(kBlock) k_request_begin(InstDesc *const *descs, float tau_unused) {
  const InstDesc &D = inst(descs);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j < sld(D.n)) sld(D.f)[j] = 0.f;
  if (blockIdx.x == 0 && threadIdx.x < SC_COUNT) {
    sld(D.sc)[threadIdx.x] = (threadIdx.x == SC_LAMBDA) ? sqrt(sld(D.tau)) : 0.0;
  }
  (void)tau_unused;
}

// u = g, partial ||g||^2 (first step of Algorithm 2).
__global__ void __launch_bounds__(kBlock) k_copy_g_u(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_outer(D)) return;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < sld(D.m)) {
    const float gj = sld(D.g)[j];
    sld(D.u)[j] = gj;
    dot = (double)gj * (double)gj;
  }
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

// Deterministic sum of the partials, then the scalar recurrences. One block per instance;
// np.n > 0: instance np.inst[k] (block k) has np.count[k] partials, else every instance nparts.
__global__ void __launch_bounds__(kBlock) k_finalize(InstDesc *const *descs, int nparts, int what,
                                                    Rag np) {
  const int bi = np.n ? np.inst[blockIdx.y] : (int)blockIdx.y;
  if (np.n) nparts = np.count[blockIdx.y];
  fin_block(*descs[bi], nparts, what);
}

// Initialisation of the update vectors: w = v / alpha_1, f = 0.
__global__ void __launch_bounds__(kBlock) k_init_wf(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= sld(D.n)) return;
  if (sld(D.sc)[SC_HALT] != 0.0) return;   // keep the f of the last outer step run
  const bool stop = sld(D.sc)[SC_STOP] != 0.0;
  sld(D.f)[j] = 0.f;
  sld(D.w)[j] = stop ? 0.f : (float)sld(D.sc)[SC_SV] * sld(D.v)[j];
}

// f += (phi/rho) w ; w = v/alpha - (theta/rho) w  (Algorithm 2, update step); 4 voxels
// per thread when n is a multiple of 4.
// pending_only: only an update left pending by the last step (see SC_UPD).
__global__ void __launch_bounds__(kBlock) k_update_fw(InstDesc *const *descs, int pending_only,
                                                     Rag rg) {
  const Blk k = locate(rg);
  if (k.i < 0) return;
  const InstDesc &D = *descs[k.i];
  const double *sc = sld(D.sc);
  if (sc[SC_STOP] != 0.0) return;
  if (pending_only && sc[SC_UPD] == 0.0) return;
  const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW], sv = (float)sc[SC_SV];
  const long long t = (long long)k.bx * kBlock + threadIdx.x;
  if ((sld(D.n) & 3) == 0) {
    if (t * 4 >= sld(D.n)) return;
    float4 wv = reinterpret_cast<const float4 *>(sld(D.w))[t];
    float4 fv = reinterpret_cast<const float4 *>(sld(D.f))[t];
    const float4 vv = reinterpret_cast<const float4 *>(sld(D.v))[t];
    fv.x += cf * wv.x; fv.y += cf * wv.y; fv.z += cf * wv.z; fv.w += cf * wv.w;
    wv.x = sv * vv.x - cw * wv.x; wv.y = sv * vv.y - cw * wv.y;
    wv.z = sv * vv.z - cw * wv.z; wv.w = sv * vv.w - cw * wv.w;
    reinterpret_cast<float4 *>(sld(D.f))[t] = fv;
    reinterpret_cast<float4 *>(sld(D.w))[t] = wv;
  } else {
    for (long long j = t * 4; j < t * 4 + 4 && j < sld(D.n); ++j) {
      const float wj = sld(D.w)[j];
      sld(D.f)[j] += cf * wj;
      sld(D.w)[j] = sv * sld(D.v)[j] - cw * wj;
    }
  }
}

// S4 residual by recurrence (Section 3.4 with the relations of the bidiagonalisation).
// With u_raw = beta_{i+1} u_{i+1} = A v_i - alpha_i u_i (the stored, unnormalised u):
//   A w_i     = u_raw + s_i,  s_i = alpha_i u_i - (theta_i / rho_{i-1}) A w_{i-1}  (s_1 = alpha_1 u_1)
//   A f_i     = A f_{i-1} + (phi_i / rho_i) A w_i
//   s_{i+1}   = alpha_{i+1} u_{i+1} - (theta_{i+1} / rho_i) A w_i
// so ||g - A f_i|| needs no product with A. aw holds s_i, af holds A f_i (n_Y each).
__global__ void __launch_bounds__(kBlock) k_s4_begin(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= sld(D.m)) return;
  const double *sc = sld(D.sc);
  if (sc[SC_STOP] != 0.0) return;
  const float c = (float)(sc[SC_ALPHA] * sc[SC_SU]);
  sld(D.aw)[j] = c * sld(D.u)[j];
  sld(D.af)[j] = 0.f;
}

__global__ void __launch_bounds__(kBlock) k_s4_step(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  const double *sc = sld(D.sc);
  if (sc[SC_STOP] != 0.0) return;   // uniform over the block: no partial is read after a stop
  const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW];
  const float cu = (float)(sc[SC_ALPHA] * sc[SC_SU]);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < sld(D.m)) {
    float *aw = sld(D.aw), *af = sld(D.af);
    const float u = sld(D.u)[j];
    const float z = u + aw[j];
    const float q = af[j] + cf * z;
    af[j] = q;
    aw[j] = cu * u - cw * z;
    const double r = (double)sld(D.g)[j] - (double)q;
    dot = r * r;
  }
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

// ------------------------------------------------------------------------------------
// Several dampings from one Krylov run (Section 3.3): the bidiagonalisation of the last outer
// step does not depend on tau, so its vectors v_1.. (scaled to the normalised v of
// Algorithm 2) are kept, and for each tau the projected problem (3.6) is solved and f(tau)
// formed from them.
// ------------------------------------------------------------------------------------
// v_{i+1} (after step i; v_1 after the initialisation) into basis slot i, last outer step only.
__global__ void __launch_bounds__(kBlock) k_basis_store(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  float *basis = sld(D.basis);
  const double *sc = sld(D.sc);
  if (!basis || sc[SC_STOP] != 0.0) return;
  if ((int)sc[SC_OUTER] != sld(D.outer_count)) return;
  const int slot = (int)sc[SC_DONE];
  if (slot >= sld(D.inner_count)) return;
  const long long n = sld(D.n);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  basis[(long long)slot * n + j] = (float)sc[SC_SV] * sld(D.v)[j];
}

// y(tau_t) for thread t: the damped QR of [B_k; sqrt(tau) I] by the rotations of Algorithm 2
// with the damping of Section 3.3 (FP64, over the k = SC_DONE completed steps), then the
// bidiagonal back substitution R y = phi; stored as float coefficients of v_1..v_k.
__global__ void __launch_bounds__(kBlock) k_tau_solve(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  const int t = threadIdx.x;
  if (t >= sld(D.n_tau) || !sld(D.basis)) return;
  const double *sc = sld(D.sc);
  const int inner = sld(D.inner_count);
  const int k = sc[SC_STATUS] != 0.0 ? 0 : (int)sc[SC_DONE];
  const double *ha = sld(D.hist), *hb = ha + inner + 1;
  double *scr = sld(D.tau_scr) + (long long)t * inner * 3;   // rho, theta, phi per step
  float *y = sld(D.ycoef) + (long long)t * inner;
  const double lam = sqrt(sld(D.taus[t]));
  double rhobar = ha[0], phibar = hb[0];
  for (int i = 1; i <= k; ++i) {
    const double beta = hb[i], alpha = ha[i];
    const double rhohat = hypot(rhobar, lam);
    phibar = (rhobar / rhohat) * phibar;
    const double rho = hypot(rhohat, beta);
    const double c = rhohat / rho, s = beta / rho;
    scr[3 * (i - 1)] = rho;
    scr[3 * (i - 1) + 1] = s * alpha;   // theta_{i+1}
    scr[3 * (i - 1) + 2] = c * phibar;  // phi_i
    rhobar = -c * alpha;
    phibar = s * phibar;
  }
  double next = 0.0;
  for (int i = k; i >= 1; --i) {
    const double rho = scr[3 * (i - 1)], phi = scr[3 * (i - 1) + 2];
    const double theta = i < k ? scr[3 * (i - 1) + 1] : 0.0;
    next = (phi - theta * next) / rho;
    y[i - 1] = (float)next;
  }
}

// f(tau_t)[j] = sum_{i < k} y_t[i] v_i[j] for up to 8 dampings per pass (coefficients in LDS,
// the basis read once per pass); written to the caller's rows only if the request succeeded.
constexpr int kTauPass = 8;
__global__ void __launch_bounds__(kBlock) k_tau_combine(InstDesc *const *descs, int t0) {
  const InstDesc &D = inst(descs);
  __shared__ float ys[kTauPass * kMaxTauInner];
  const double *sc = sld(D.sc);
  if (!sld(D.basis) || sc[SC_STATUS] != 0.0) return;
  const int inner = sld(D.inner_count);
  const int k = (int)sc[SC_DONE];
  const int nt = min(kTauPass, sld(D.n_tau) - t0);
  if (nt <= 0) return;
  const float *y = sld(D.ycoef);
  for (int q = threadIdx.x; q < nt * k; q += kBlock)
    ys[q] = y[(long long)(t0 + q / k) * inner + q % k];
  __syncthreads();
  const long long n = sld(D.n);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const float *basis = sld(D.basis);
  float acc[kTauPass];
#pragma unroll
  for (int t = 0; t < kTauPass; ++t) acc[t] = 0.f;
  for (int i = 0; i < k; ++i) {
    const float b = basis[(long long)i * n + j];
#pragma unroll
    for (int t = 0; t < kTauPass; ++t)
      if (t < nt) acc[t] += ys[t * k + i] * b;
  }
  float *out = sld(D.f_taus);
#pragma unroll
  for (int t = 0; t < kTauPass; ++t)
    if (t < nt) out[(long long)(t0 + t) * n + j] = acc[t];
}

// partial of v . p (alpha^2 when the V-cycle is a single exact solve)
__global__ void __launch_bounds__(kBlock) k_dot_vp(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (j < sld(D.n)) dot = (double)sld(D.v)[j] * (double)sld(D.p)[j];
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

// Copy f^K to the caller's buffer if the request succeeded.
__global__ void __launch_bounds__(kBlock) k_copy_out(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= sld(D.n)) return;
  if (sld(D.sc)[SC_STATUS] != 0.0) return;
  sld(D.out_f)[j] = sld(D.f)[j];
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

#define LAUNCH(kern, gx, gy, ...) \
  hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kBlock), 0, st, __VA_ARGS__)

void launch_request_begin(hipStream_t st, InstDesc *const *d, int B, long long n) {
  LAUNCH(k_request_begin, blocks_for(n), B, d, 0.f);
}
void launch_outer_begin(hipStream_t st, InstDesc *const *d, int B) {
  hipLaunchKernelGGL(k_outer_begin, dim3(1, B), dim3(64), 0, st, d, 0);
}
int launch_diffusivity(hipStream_t st, InstDesc *const *d, int B, long long n, int write_kappa) {
  const unsigned g = blocks_for(n);
  LAUNCH(k_diffusivity, g, B, d, write_kappa);
  return (int)g;
}
void launch_level0_dinv(hipStream_t st, InstDesc *const *d, int B, long long n) {
  LAUNCH(k_level0_dinv, blocks_for(n), B, d);
}
void launch_coarsen(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse) {
  LAUNCH(k_coarsen, blocks_for(n_coarse), B, d, l);
}
void launch_level_dinv(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l) {
  LAUNCH(k_level_dinv, blocks_for(n_l), B, d, l);
}
void launch_coarse_factor(hipStream_t st, InstDesc *const *d, int B) {
  LAUNCH(k_coarse_factor, 1, B, d);
}
void launch_coarse_solve(hipStream_t st, InstDesc *const *d, int B) {
  LAUNCH(k_coarse_solve, 1, B, d);
}
int launch_jacobi(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int first,
                  int src, int dst, int want_dot) {
  const unsigned g = blocks_for(n_l);
  LAUNCH(k_jacobi, g, B, d, l, first, src, dst, want_dot);
  return (int)g;
}
void launch_cheb_start(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int zero_x,
                       int d_sel) {
  LAUNCH(k_cheb_start, blocks_for(n_l), B, d, l, zero_x, d_sel);
}
int launch_cheb_step(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int set_x,
                     int update_r, int last, int d_sel, int dn_sel, int step, int want_dot,
                     int add_prolong) {
  const unsigned g = blocks_for(n_l);
  LAUNCH(k_cheb_step, g, B, d, l, set_x, update_r, last, d_sel, dn_sel, step, want_dot,
         add_prolong);
  return (int)g;
}
int launch_jacobi_first2(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int dst,
                         int want_dot) {
  const unsigned g = blocks_for(n_l);
  LAUNCH(k_jacobi_first2, g, B, d, l, dst, want_dot);
  return (int)g;
}
int launch_jacobi_prolong(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int src,
                          int dst, int want_dot) {
  const unsigned g = blocks_for(n_l);
  LAUNCH(k_jacobi_prolong, g, B, d, l, src, dst, want_dot);
  return (int)g;
}
void launch_cheb_first(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int last,
                       int dn_sel) {
  LAUNCH(k_cheb_first, blocks_for(n_l), B, d, l, last, dn_sel);
}
void launch_cheb_start_prolong(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l,
                               int d_sel) {
  LAUNCH(k_cheb_start_prolong, blocks_for(n_l), B, d, l, d_sel);
}
void launch_restrict_fine(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse,
                          int nchild, int x_sel, int use_r) {
  LAUNCH(k_restrict_fine, blocks_for(n_coarse * nchild), B, d, l, x_sel, use_r);
}
int launch_copy_g_u(hipStream_t st, InstDesc *const *d, int B, long long m) {
  const unsigned g = blocks_for(m);
  LAUNCH(k_copy_g_u, g, B, d);
  return (int)g;
}
void launch_finalize(hipStream_t st, InstDesc *const *d, int B, int nparts, int what,
                     const Rag &np) {
  LAUNCH(k_finalize, 1, np.n ? np.n : B, d, nparts, what, np);
}
void launch_init_wf(hipStream_t st, InstDesc *const *d, int B, long long n) {
  LAUNCH(k_init_wf, blocks_for(n), B, d);
}
void launch_update_fw(hipStream_t st, InstDesc *const *d, int B, long long n, const Rag &rg,
                      int pending_only) {
  if (rg.n == 0) {
    LAUNCH(k_update_fw, blocks_for((n + 3) / 4), B, d, pending_only, rg);
  } else {
    const unsigned g = (unsigned)(rg.first[rg.n - 1] + rg.count[rg.n - 1]);
    LAUNCH(k_update_fw, g, 1, d, pending_only, rg);
  }
}
int launch_dot_vp(hipStream_t st, InstDesc *const *d, int B, long long n) {
  const unsigned g = blocks_for(n);
  LAUNCH(k_dot_vp, g, B, d);
  return (int)g;
}
void launch_s4_begin(hipStream_t st, InstDesc *const *d, int B, long long m) {
  LAUNCH(k_s4_begin, blocks_for(m), B, d);
}
int launch_s4_step(hipStream_t st, InstDesc *const *d, int B, long long m) {
  const unsigned g = blocks_for(m);
  LAUNCH(k_s4_step, g, B, d);
  return (int)g;
}
void launch_basis_store(hipStream_t st, InstDesc *const *d, int B, long long n) {
  LAUNCH(k_basis_store, blocks_for(n), B, d);
}
void launch_tau_finish(hipStream_t st, InstDesc *const *d, int B, long long n, int n_tau) {
  LAUNCH(k_tau_solve, 1, B, d);
  for (int t0 = 0; t0 < n_tau; t0 += kTauPass) LAUNCH(k_tau_combine, blocks_for(n), B, d, t0);
}
void launch_copy_out(hipStream_t st, InstDesc *const *d, int B, long long n) {
  LAUNCH(k_copy_out, blocks_for(n), B, d);
}

}  // namespace plsqr
