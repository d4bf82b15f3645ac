// V-cycle tail with its levels resident in LDS: every level from `t` (>= 1) down to the
// coarsest and back up, in one workgroup of kTailBlock threads per instance (section 4.2).
//
// The small coarse levels of a V-cycle are bound by dependency latency: a pass over 4096 cells
// or fewer is a few instructions per thread, and what it costs is the round trip of its memory
// accesses and the barrier after it. Here every vector of every tail level (iterate, right-hand
// side, residual, Chebyshev directions) and every face weight live in LDS for the whole tail,
// so a pass costs LDS latency only: the face weights and level t's right-hand side are read
// from global memory once at the start, level t's iterate is written once at the end, and the
// coarsest solve reads the FP64 inverse formed at setup.
//
// LDS is addressed only through the file-scope __shared__ arrays below, by integer offsets
// (a level's arrays are slices of one pool at offsets computed in registers); no LDS address is
// ever stored in a structure or handed to code that also handles global pointers.
//
// Each voxel's arithmetic is that of the one-pass kernels and of k_vcycle_tail (the same terms
// in the same order; 1/diag is formed in the order of the stored coarse diagonals), so the two
// tails give the same values.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

__shared__ float tpool[kTailLdsFloats];
__shared__ double tbs[PLSQR_MAX_COARSE];

// Arrays of a tail level, as slices of tpool: vectors first, then the face weights.
enum TailArr : int { TA_X = 0, TA_B, TA_R, TA_DA, TA_DB, TA_WX, TA_WY, TA_WZ, TA_COUNT };

struct TailLevel {
  int nx, ny, nz, n;
  int base;          // offset of the level's first array in tpool
  float eps;
};

__device__ __forceinline__ int ti(const TailLevel &g, int a, int j) { return g.base + a * g.n + j; }

// (A_l x)_j for x in array `a` of level g (levels >= 1: stored face weights), terms in the order
// of the one-pass stencil.
__device__ __forceinline__ float tstencil(const TailLevel &g, int a, int j, int x, int y, int z) {
  const int sy = g.nx, sz = g.nx * g.ny;
  const float xj = tpool[ti(g, a, j)];
  float acc = g.eps * xj;
  if (x + 1 < g.nx) acc += tpool[ti(g, TA_WX, j)] * (xj - tpool[ti(g, a, j + 1)]);
  if (x > 0) acc += tpool[ti(g, TA_WX, j - 1)] * (xj - tpool[ti(g, a, j - 1)]);
  if (y + 1 < g.ny) acc += tpool[ti(g, TA_WY, j)] * (xj - tpool[ti(g, a, j + sy)]);
  if (y > 0) acc += tpool[ti(g, TA_WY, j - sy)] * (xj - tpool[ti(g, a, j - sy)]);
  if (g.nz > 1) {
    if (z + 1 < g.nz) acc += tpool[ti(g, TA_WZ, j)] * (xj - tpool[ti(g, a, j + sz)]);
    if (z > 0) acc += tpool[ti(g, TA_WZ, j - sz)] * (xj - tpool[ti(g, a, j - sz)]);
  }
  return acc;
}

// 1/diag_j in the order of the stored coarse diagonal: eps, then each axis's pair of faces.
__device__ __forceinline__ float tdinv(const TailLevel &g, int j, int x, int y, int z) {
  const int sy = g.nx, sz = g.nx * g.ny;
  float d = g.eps;
  d += tpool[ti(g, TA_WX, j)] + (x > 0 ? tpool[ti(g, TA_WX, j - 1)] : 0.f);
  d += tpool[ti(g, TA_WY, j)] + (y > 0 ? tpool[ti(g, TA_WY, j - sy)] : 0.f);
  if (g.nz > 1) d += tpool[ti(g, TA_WZ, j)] + (z > 0 ? tpool[ti(g, TA_WZ, j - sz)] : 0.f);
  return 1.0f / d;
}

// One pass over the cells of a level, then a barrier. body(j, x, y, z).
template <class F>
__device__ __forceinline__ void tpass(const TailLevel &g, F body) {
  for (int j = threadIdx.x; j < g.n; j += kTailBlock) {
    const int q = j / g.nx;
    body(j, j - q * g.nx, q % g.ny, q / g.ny);
  }
  __syncthreads();
}

__device__ __forceinline__ void cheb_coef(const InstDesc &D, int step, float &c_dd, float &c_dr) {
  double rho = 1.0 / sld(D.cheb_sigma);
  for (int i = 0; i < step; ++i) rho = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  const double rho_next = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  c_dd = (float)(rho_next * rho);
  c_dr = (float)(2.0 * rho_next / sld(D.cheb_delta));
}

// Restriction of the residual in array TA_R of level g into the right-hand side of level c:
// the children of each coarse cell summed in the order of the one-pass restriction (for each
// fine plane, each row pair in y, each row's pair in x).
__device__ __forceinline__ void trestrict(const TailLevel &g, const TailLevel &c) {
  const int cz = (g.nz > 1) ? 2 : 1;
  tpass(c, [&](int J, int cx, int cy, int czc) {
    float s = 0.f;
    for (int dz = 0; dz < cz; ++dz)
      for (int dy = 0; dy < 2; ++dy) {
        const int jf = 2 * cx + g.nx * ((2 * cy + dy) + g.ny * (cz * czc + dz));
        s += tpool[ti(g, TA_R, jf)];
        s += tpool[ti(g, TA_R, jf + 1)];
      }
    tpool[ti(c, TA_B, J)] = s;
  });
}

// x_l += P x_{l+1} (pointwise): every fine cell of array xa takes its coarse parent's value from
// the coarse level's array ca.
__device__ __forceinline__ void tprolong(const TailLevel &g, int xa, const TailLevel &c, int ca) {
  const int cz = (g.nz > 1) ? 2 : 1;
  tpass(g, [&](int j, int x, int y, int z) {
    const int p = (x >> 1) + c.nx * ((y >> 1) + c.ny * (z / cz));
    tpool[ti(g, xa, j)] += tpool[ti(c, ca, p)];
  });
}

// Tail level l (>= t) from the descriptor (uniform scalar loads): its pool slice follows those of
// levels t .. l - 1.
__device__ __forceinline__ TailLevel tail_level(const InstDesc &D, int t, int l) {
  TailLevel g;
  int off = 0;
  for (int k = t; k < l; ++k) off += TA_COUNT * (int)sld(D.lv[k].n);
  g.nx = sld(D.lv[l].nx);
  g.ny = sld(D.lv[l].ny);
  g.nz = sld(D.lv[l].nz);
  g.n = (int)sld(D.lv[l].n);
  g.eps = (float)sld(D.lv[l].eps);
  g.base = off;
  return g;
}

}  // namespace

__global__ void __launch_bounds__(kTailBlock) k_vcycle_tail_lds(InstDesc *const *descs, int t) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const int Lv = sld(D.levels);
  const int nu = sld(D.nu_pre);
  // the face weights of every tail level and level t's right-hand side
  for (int l = t; l < Lv; ++l) {
    const LevelDesc L = level_of(D, l);
    const TailLevel g = tail_level(D, t, l);
    const bool hz = g.nz > 1;
    for (int j = threadIdx.x; j < g.n; j += kTailBlock) {
      tpool[ti(g, TA_WX, j)] = L.wx[j];
      tpool[ti(g, TA_WY, j)] = L.wy[j];
      tpool[ti(g, TA_WZ, j)] = hz ? L.wz[j] : 0.f;
      if (l == t) tpool[ti(g, TA_B, j)] = L.b[j];
    }
  }
  __syncthreads();
  const float om = sld(D.omega);
  const bool jac = sld(D.smoother) == PLSQR_SMOOTH_JACOBI;
  const int m = sld(D.cheb_degree);
  const float ith = jac ? 0.f : (float)(1.0 / sld(D.cheb_theta));
  // Jacobi: the current iterate alternates between TA_X and TA_DA (bit l of in_da: level l's
  // iterate is in TA_DA)
  unsigned in_da = 0;

  // ---- down ------------------------------------------------------------------------------
  for (int l = t; l < Lv - 1; ++l) {
    const TailLevel g = tail_level(D, t, l);
    if (jac) {
      // x1 = omega D^{-1} b, then nu - 1 sweeps x <- x + omega D^{-1} (b - A x), then r = b - A x
      tpass(g, [&](int j, int x, int y, int z) {
        tpool[ti(g, TA_X, j)] = om * tdinv(g, j, x, y, z) * tpool[ti(g, TA_B, j)];
      });
      int cur = TA_X;
      for (int s = 1; s < nu; ++s) {
        const int nxt = (cur == TA_X) ? TA_DA : TA_X;
        tpass(g, [&](int j, int x, int y, int z) {
          const float ax = tstencil(g, cur, j, x, y, z);
          tpool[ti(g, nxt, j)] = tpool[ti(g, cur, j)] +
                                 om * tdinv(g, j, x, y, z) * (tpool[ti(g, TA_B, j)] - ax);
        });
        cur = nxt;
      }
      if (cur == TA_DA) in_da |= 1u << l;
      tpass(g, [&](int j, int x, int y, int z) {
        tpool[ti(g, TA_R, j)] = tpool[ti(g, TA_B, j)] - tstencil(g, cur, j, x, y, z);
      });
    } else {
      for (int a = 0; a < nu; ++a) {
        int dcur = TA_DA;
        int k0 = 0;
        if (a == 0) {
          // start and first step from x = 0: x = d0 = D^{-1} b / theta, r = b - A d0, d1
          float c_dd, c_dr;
          cheb_coef(D, 0, c_dd, c_dr);
          tpass(g, [&](int j, int x, int y, int z) {
            tpool[ti(g, TA_X, j)] = ith * tdinv(g, j, x, y, z) * tpool[ti(g, TA_B, j)];
          });
          const bool last = (m == 1);
          tpass(g, [&](int j, int x, int y, int z) {
            const float d0 = tpool[ti(g, TA_X, j)];
            const float r = tpool[ti(g, TA_B, j)] - tstencil(g, TA_X, j, x, y, z);
            tpool[ti(g, TA_R, j)] = r;
            if (!last) tpool[ti(g, TA_DA, j)] = c_dd * d0 + c_dr * tdinv(g, j, x, y, z) * r;
          });
          k0 = 1;
        } else {
          // r = b - A x, d = D^{-1} r / theta
          tpass(g, [&](int j, int x, int y, int z) {
            const float r = tpool[ti(g, TA_B, j)] - tstencil(g, TA_X, j, x, y, z);
            tpool[ti(g, TA_R, j)] = r;
            tpool[ti(g, TA_DA, j)] = ith * tdinv(g, j, x, y, z) * r;
          });
        }
        for (int k = k0; k < m; ++k) {
          const bool last = (k == m - 1);
          const bool upd = !last || (a == nu - 1);
          const int dn = (dcur == TA_DA) ? TA_DB : TA_DA;
          float c_dd, c_dr;
          cheb_coef(D, k, c_dd, c_dr);
          tpass(g, [&](int j, int x, int y, int z) {
            const float dj = tpool[ti(g, dcur, j)];
            tpool[ti(g, TA_X, j)] = tpool[ti(g, TA_X, j)] + dj;
            if (upd) {
              const float r = tpool[ti(g, TA_R, j)] - tstencil(g, dcur, j, x, y, z);
              tpool[ti(g, TA_R, j)] = r;
              if (!last) tpool[ti(g, dn, j)] = c_dd * dj + c_dr * tdinv(g, j, x, y, z) * r;
            }
          });
          dcur = dn;
        }
      }
    }
    trestrict(g, tail_level(D, t, l + 1));
  }

  // ---- coarsest: x = A_c^{-1} b with the FP64 inverse, each row split over a group of lanes --
  {
    const TailLevel g = tail_level(D, t, Lv - 1);
    const int n = g.n;
    const double *__restrict__ Ai = sld(D.cfac) + (long long)n * n * 2;
    for (int i = threadIdx.x; i < n; i += kTailBlock) tbs[i] = (double)tpool[ti(g, TA_B, i)];
    __syncthreads();
    int gl = 1;   // lanes per row: the largest power of two <= min(64, kTailBlock / n)
    while (2 * gl <= 64 && 2 * gl * n <= kTailBlock) gl *= 2;
    const int s = threadIdx.x % gl;
    const int rows_per_pass = kTailBlock / gl;
    for (int i0 = 0; i0 < n; i0 += rows_per_pass) {
      const int i = i0 + (int)threadIdx.x / gl;
      double acc = 0.0;
      if (i < n)
        for (int jj = s; jj < n; jj += gl) acc += Ai[(long long)jj * n + i] * tbs[jj];
      for (int o = 1; o < gl; o <<= 1) acc += __shfl_xor(acc, o, 64);
      if (i < n && s == 0) tpool[ti(g, TA_X, i)] = (float)acc;
    }
    __syncthreads();
  }

  // ---- up ----------------------------------------------------------------------------------
  for (int l = Lv - 2; l >= t; --l) {
    const TailLevel g = tail_level(D, t, l);
    const TailLevel c = tail_level(D, t, l + 1);
    if (jac) {
      // the coarse level's iterate: the coarsest solve writes TA_X, a smoothed level the array
      // its last sweep wrote
      int cur = ((in_da >> l) & 1u) ? TA_DA : TA_X;
      tprolong(g, cur, c, ((in_da >> (l + 1)) & 1u) ? TA_DA : TA_X);
      for (int s = 0; s < nu; ++s) {
        const int nxt = (cur == TA_X) ? TA_DA : TA_X;
        tpass(g, [&](int j, int x, int y, int z) {
          const float ax = tstencil(g, cur, j, x, y, z);
          tpool[ti(g, nxt, j)] = tpool[ti(g, cur, j)] +
                                 om * tdinv(g, j, x, y, z) * (tpool[ti(g, TA_B, j)] - ax);
        });
        cur = nxt;
      }
      in_da = (in_da & ~(1u << l)) | ((cur == TA_DA ? 1u : 0u) << l);
    } else {
      tprolong(g, TA_X, c, TA_X);
      for (int a = 0; a < nu; ++a) {
        // r = b - A x, d = D^{-1} r / theta (the first time on x + P e)
        tpass(g, [&](int j, int x, int y, int z) {
          const float r = tpool[ti(g, TA_B, j)] - tstencil(g, TA_X, j, x, y, z);
          tpool[ti(g, TA_R, j)] = r;
          tpool[ti(g, TA_DA, j)] = ith * tdinv(g, j, x, y, z) * r;
        });
        int dcur = TA_DA;
        for (int k = 0; k < m; ++k) {
          const bool last = (k == m - 1);
          const int dn = (dcur == TA_DA) ? TA_DB : TA_DA;
          float c_dd, c_dr;
          cheb_coef(D, k, c_dd, c_dr);
          tpass(g, [&](int j, int x, int y, int z) {
            const float dj = tpool[ti(g, dcur, j)];
            tpool[ti(g, TA_X, j)] = tpool[ti(g, TA_X, j)] + dj;
            if (!last) {
              const float r = tpool[ti(g, TA_R, j)] - tstencil(g, dcur, j, x, y, z);
              tpool[ti(g, TA_R, j)] = r;
              tpool[ti(g, dn, j)] = c_dd * dj + c_dr * tdinv(g, j, x, y, z) * r;
            }
          });
          dcur = dn;
        }
      }
    }
  }
  // level t's iterate back to global memory for the level above
  {
    const LevelDesc L = level_of(D, t);
    const TailLevel g = tail_level(D, t, t);
    const int a = (jac && ((in_da >> t) & 1u)) ? TA_DA : TA_X;
    for (int j = threadIdx.x; j < g.n; j += kTailBlock) L.x[j] = tpool[ti(g, a, j)];
  }
}

long long tail_lds_floats(const long long *cells, int nlev) {
  long long s = 0;
  for (int i = 0; i < nlev; ++i) s += (long long)TA_COUNT * cells[i];
  return s;
}

void launch_vcycle_tail_lds(hipStream_t st, InstDesc *const *d, int B, int t) {
  hipLaunchKernelGGL(k_vcycle_tail_lds, dim3(1, B), dim3(kTailBlock), 0, st, d, t);
}

}  // namespace plsqr
