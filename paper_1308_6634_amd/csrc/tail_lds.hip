// V-cycle tail with its levels resident in LDS: every level from `t` (>= 1) down to the
// coarsest and back up, in one workgroup of kTailBlock threads per instance (section 4.2).
//
// The small coarse levels of a V-cycle are bound by dependency latency: a pass over 4096 cells
// or fewer is a few instructions per thread, and what it costs is the round trip of its memory
// accesses and the barrier after it. Here every vector of every tail level (iterate, right-hand
// side, residual, Chebyshev directions) and every face weight live in LDS for the whole tail,
// so a pass costs LDS latency only: the face weights and level t's right-hand side are read
// from global memory once at the start, and level t's iterate is written once at the end.
//
// On entering a level each thread forms, for the cells it owns, 1/diag and the six face
// weights (zero where a face has no neighbour) in registers; a pass then reads only the vectors
// it combines. A pass first reads everything its cells need and computes their results, then
// stores them: no pass writes an array that it reads at a neighbour, so the loads of all of a
// thread's cells are issued back to back.
//
// LDS is addressed only through the file-scope __shared__ arrays below, by integer offsets
// (a level's arrays are slices of one pool at offsets computed in registers); no LDS address is
// ever stored in a structure or handed to code that also handles global pointers.
//
// Each voxel's arithmetic is that of the one-pass kernels and of k_vcycle_tail (the same terms
// in the same order; 1/diag is formed in the order of the stored coarse diagonals; a face
// without a neighbour adds 0 * (x_j - x_k) for some in-range k, which leaves the sum unchanged),
// so the two tails give the same values.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

__shared__ float tpool[kTailLdsFloats];
__shared__ double tbs[PLSQR_MAX_COARSE];
__shared__ float tcdd[kMaxChebDegree], tcdr[kMaxChebDegree];   // Chebyshev step coefficients

// Arrays of a tail level, as slices of tpool: vectors first, then the face weights.
enum TailArr : int { TA_X = 0, TA_B, TA_R, TA_DA, TA_DB, TA_WX, TA_WY, TA_WZ, TA_COUNT };

// Most cells one thread owns on a tail level (the host admits levels of at most
// kTailMaxPer * kTailBlock cells).
static_assert(kTailMaxPer == 4, "the level dispatch below covers 1 to 4 cells per thread");
// FP64 entries of the coarsest inverse a thread holds in registers when its rows fit one pass.
constexpr int kTailAi = 8;

struct TailLevel {
  int nx, ny, nz, n;
  int base;          // offset of the level's first array in tpool
  float eps;
};

__device__ __forceinline__ int ti(const TailLevel &g, int a, int j) { return g.base + a * g.n + j; }

// The cells a thread owns on one level: slot k is cell threadIdx.x + k kTailBlock, the last slot
// clamped to the level's last cell (its results are stored only when it is a cell of its own),
// so that every slot's loads are unconditional. aux: on the way down the first fine child of
// the cell (restriction), on the way up its coarse parent (prolongation).
__device__ __forceinline__ int tj(const TailLevel &g, int k) {
  return min((int)threadIdx.x + k * kTailBlock, g.n - 1);
}
template <int P>
struct TCells {
  int aux[P];
  float dinv[P];
  float wxp[P], wxm[P], wyp[P], wym[P], wzp[P], wzm[P];
  bool last_real;
};

// Cells of level g. f: the next finer level (aux on the way down), c: the next coarser level
// (aux on the way up); `smooth`: whether the weights and 1/diag are needed (not on the
// coarsest level).
template <int P>
__device__ __forceinline__ void tcells(const TailLevel &g, const TailLevel &f, const TailLevel &c,
                                       bool down, bool smooth, TCells<P> &s) {
  const int sy = g.nx, sz = g.nx * g.ny;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int j = tj(g, k);
    const int q = j / g.nx;
    const int x = j - q * g.nx, y = q % g.ny, z = q / g.ny;
    if (down) {
      // first child on the finer level (2:1 in x and y; in z when f has several planes)
      const int fz = (f.nz > 1) ? 2 : 1;
      s.aux[k] = 2 * x + f.nx * (2 * y + f.ny * (fz * z));
    } else {
      const int cz = (g.nz > 1) ? 2 : 1;
      s.aux[k] = (x >> 1) + c.nx * ((y >> 1) + c.ny * (z / cz));
    }
    if (smooth) {
      const float wx = tpool[ti(g, TA_WX, j)], wy = tpool[ti(g, TA_WY, j)];
      const float wz = tpool[ti(g, TA_WZ, j)];
      const float wxl = tpool[ti(g, TA_WX, max(j - 1, 0))];
      const float wyl = tpool[ti(g, TA_WY, max(j - sy, 0))];
      const float wzl = tpool[ti(g, TA_WZ, max(j - sz, 0))];
      const float wxm = x > 0 ? wxl : 0.f, wym = y > 0 ? wyl : 0.f, wzm = z > 0 ? wzl : 0.f;
      float d = g.eps;
      d += wx + wxm;
      d += wy + wym;
      if (g.nz > 1) d += wz + wzm;
      s.dinv[k] = 1.0f / d;
      s.wxp[k] = (x + 1 < g.nx) ? wx : 0.f;
      s.wxm[k] = wxm;
      s.wyp[k] = (y + 1 < g.ny) ? wy : 0.f;
      s.wym[k] = wym;
      s.wzp[k] = (z + 1 < g.nz) ? wz : 0.f;
      s.wzm[k] = wzm;
    }
  }
  s.last_real = (int)threadIdx.x + (P - 1) * kTailBlock < g.n;
}

// (A_l x)_j for the cell in slot k and x in array `a` of level g, terms in the order of the
// one-pass stencil (+x, -x, +y, -y, +z, -z).
template <int P>
__device__ __forceinline__ float tA(const TailLevel &g, const TCells<P> &s, int k, int a) {
  const int o = g.base + a * g.n, j = tj(g, k), last = g.n - 1;
  const int sy = g.nx, sz = g.nx * g.ny;
  const float xj = tpool[o + j];
  float acc = g.eps * xj;
  acc += s.wxp[k] * (xj - tpool[o + min(j + 1, last)]);
  acc += s.wxm[k] * (xj - tpool[o + max(j - 1, 0)]);
  acc += s.wyp[k] * (xj - tpool[o + min(j + sy, last)]);
  acc += s.wym[k] * (xj - tpool[o + max(j - sy, 0)]);
  acc += s.wzp[k] * (xj - tpool[o + min(j + sz, last)]);
  acc += s.wzm[k] * (xj - tpool[o + max(j - sz, 0)]);
  return acc;
}

// One pass: compute(k) for every slot, then store(k, value) for the thread's own cells, then a
// barrier.
template <int P, class C, class S>
__device__ __forceinline__ void tpass(const TCells<P> &s, C compute, S store) {
  decltype(compute(0)) v[P];
#pragma unroll
  for (int k = 0; k < P; ++k) v[k] = compute(k);
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (k < P - 1 || s.last_real) store(k, v[k]);
  __syncthreads();
}

struct F2 { float a, b; };
struct F3 { float a, b, c; };

__device__ __forceinline__ void cheb_coef(const InstDesc &D, int step, float &c_dd, float &c_dr) {
  double rho = 1.0 / sld(D.cheb_sigma);
  for (int i = 0; i < step; ++i) rho = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  const double rho_next = 1.0 / (2.0 * sld(D.cheb_sigma) - rho);
  c_dd = (float)(rho_next * rho);
  c_dr = (float)(2.0 * rho_next / sld(D.cheb_delta));
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

__device__ __forceinline__ int tail_per(int n) { return (n + kTailBlock - 1) / kTailBlock; }

// Smoother parameters shared by every level.
struct TailSm {
  bool jac;
  int nu, m;
  float om, ith;
};

// Down leg of level g: (when restrict_in) the restriction of the finer level f's residual into
// b_g, then (when smooth) the pre-smoothing from x = 0 and the residual r = b - A x. Returns
// whether the Jacobi iterate ended in TA_DA.
template <int P>
__device__ bool tail_down(const InstDesc &D, const TailSm &m, const TailLevel &f,
                          const TailLevel &g, bool restrict_in, bool smooth) {
  TCells<P> s;
  tcells<P>(g, f, g, true, smooth, s);
  if (restrict_in) {
    // b[J] = the children of J summed in the order of the one-pass restriction (for each fine
    // plane, each row pair in y, each row's pair in x)
    const int fz = (f.nz > 1) ? 2 : 1;
    tpass<P>(s, [&](int k) {
      float acc = 0.f;
      for (int dz = 0; dz < fz; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
          const int jf = s.aux[k] + f.nx * (dy + f.ny * dz);
          acc += tpool[ti(f, TA_R, jf)];
          acc += tpool[ti(f, TA_R, jf + 1)];
        }
      return acc;
    }, [&](int k, float v) { tpool[ti(g, TA_B, tj(g, k))] = v; });
  }
  if (!smooth) return false;
  if (m.jac) {
    // x1 = omega D^{-1} b, then nu - 1 sweeps x <- x + omega D^{-1} (b - A x), then r = b - A x
    tpass<P>(s, [&](int k) { return m.om * s.dinv[k] * tpool[ti(g, TA_B, tj(g, k))]; },
             [&](int k, float v) { tpool[ti(g, TA_X, tj(g, k))] = v; });
    int cur = TA_X;
    for (int it = 1; it < m.nu; ++it) {
      const int nxt = (cur == TA_X) ? TA_DA : TA_X;
      tpass<P>(s, [&](int k) {
        const float ax = tA<P>(g, s, k, cur);
        return tpool[ti(g, cur, tj(g, k))] + m.om * s.dinv[k] * (tpool[ti(g, TA_B, tj(g, k))] - ax);
      }, [&](int k, float v) { tpool[ti(g, nxt, tj(g, k))] = v; });
      cur = nxt;
    }
    tpass<P>(s, [&](int k) { return tpool[ti(g, TA_B, tj(g, k))] - tA<P>(g, s, k, cur); },
             [&](int k, float v) { tpool[ti(g, TA_R, tj(g, k))] = v; });
    return cur == TA_DA;
  }
  for (int a = 0; a < m.nu; ++a) {
    int dcur = TA_DA;
    int k0 = 0;
    if (a == 0) {
      // start and first step from x = 0: x = d0 = D^{-1} b / theta, r = b - A d0, d1
      const float c_dd = tcdd[0], c_dr = tcdr[0];
      tpass<P>(s, [&](int k) { return m.ith * s.dinv[k] * tpool[ti(g, TA_B, tj(g, k))]; },
               [&](int k, float v) { tpool[ti(g, TA_X, tj(g, k))] = v; });
      const bool last = (m.m == 1);
      tpass<P>(s, [&](int k) {
        const float d0 = tpool[ti(g, TA_X, tj(g, k))];
        const float r = tpool[ti(g, TA_B, tj(g, k))] - tA<P>(g, s, k, TA_X);
        return F2{r, c_dd * d0 + c_dr * s.dinv[k] * r};
      }, [&](int k, F2 v) {
        tpool[ti(g, TA_R, tj(g, k))] = v.a;
        if (!last) tpool[ti(g, TA_DA, tj(g, k))] = v.b;
      });
      k0 = 1;
    } else {
      // r = b - A x, d = D^{-1} r / theta
      tpass<P>(s, [&](int k) {
        const float r = tpool[ti(g, TA_B, tj(g, k))] - tA<P>(g, s, k, TA_X);
        return F2{r, m.ith * s.dinv[k] * r};
      }, [&](int k, F2 v) {
        tpool[ti(g, TA_R, tj(g, k))] = v.a;
        tpool[ti(g, TA_DA, tj(g, k))] = v.b;
      });
    }
    for (int st = k0; st < m.m; ++st) {
      const bool last = (st == m.m - 1);
      const bool upd = !last || (a == m.nu - 1);
      const int dn = (dcur == TA_DA) ? TA_DB : TA_DA;
      const float c_dd = tcdd[st], c_dr = tcdr[st];
      tpass<P>(s, [&](int k) {
        const float dj = tpool[ti(g, dcur, tj(g, k))];
        F3 o;
        o.a = tpool[ti(g, TA_X, tj(g, k))] + dj;
        o.b = 0.f;
        o.c = 0.f;
        if (upd) {
          o.b = tpool[ti(g, TA_R, tj(g, k))] - tA<P>(g, s, k, dcur);
          if (!last) o.c = c_dd * dj + c_dr * s.dinv[k] * o.b;
        }
        return o;
      }, [&](int k, F3 v) {
        tpool[ti(g, TA_X, tj(g, k))] = v.a;
        if (upd) {
          tpool[ti(g, TA_R, tj(g, k))] = v.b;
          if (!last) tpool[ti(g, dn, tj(g, k))] = v.c;
        }
      });
      dcur = dn;
    }
  }
  return false;
}

// Up leg of level g: x += P x_c (x_c in array ca of the coarser level c), then the
// post-smoothing. in_da: the Jacobi pre-smoothed iterate is in TA_DA. Returns whether the Jacobi
// iterate ended in TA_DA.
template <int P>
__device__ bool tail_up(const InstDesc &D, const TailSm &m, const TailLevel &g,
                        const TailLevel &c, int ca, bool in_da) {
  TCells<P> s;
  tcells<P>(g, g, c, false, true, s);
  if (m.jac) {
    int cur = in_da ? TA_DA : TA_X;
    tpass<P>(s, [&](int k) { return tpool[ti(g, cur, tj(g, k))] + tpool[ti(c, ca, s.aux[k])]; },
             [&](int k, float v) { tpool[ti(g, cur, tj(g, k))] = v; });
    for (int it = 0; it < m.nu; ++it) {
      const int nxt = (cur == TA_X) ? TA_DA : TA_X;
      tpass<P>(s, [&](int k) {
        const float ax = tA<P>(g, s, k, cur);
        return tpool[ti(g, cur, tj(g, k))] + m.om * s.dinv[k] * (tpool[ti(g, TA_B, tj(g, k))] - ax);
      }, [&](int k, float v) { tpool[ti(g, nxt, tj(g, k))] = v; });
      cur = nxt;
    }
    return cur == TA_DA;
  }
  tpass<P>(s, [&](int k) { return tpool[ti(g, TA_X, tj(g, k))] + tpool[ti(c, ca, s.aux[k])]; },
           [&](int k, float v) { tpool[ti(g, TA_X, tj(g, k))] = v; });
  for (int a = 0; a < m.nu; ++a) {
    // r = b - A x, d = D^{-1} r / theta (the first time on x + P e)
    tpass<P>(s, [&](int k) {
      const float r = tpool[ti(g, TA_B, tj(g, k))] - tA<P>(g, s, k, TA_X);
      return F2{r, m.ith * s.dinv[k] * r};
    }, [&](int k, F2 v) {
      tpool[ti(g, TA_R, tj(g, k))] = v.a;
      tpool[ti(g, TA_DA, tj(g, k))] = v.b;
    });
    int dcur = TA_DA;
    for (int st = 0; st < m.m; ++st) {
      const bool last = (st == m.m - 1);
      const int dn = (dcur == TA_DA) ? TA_DB : TA_DA;
      const float c_dd = tcdd[st], c_dr = tcdr[st];
      tpass<P>(s, [&](int k) {
        const float dj = tpool[ti(g, dcur, tj(g, k))];
        F3 o;
        o.a = tpool[ti(g, TA_X, tj(g, k))] + dj;
        o.b = 0.f;
        o.c = 0.f;
        if (!last) {
          o.b = tpool[ti(g, TA_R, tj(g, k))] - tA<P>(g, s, k, dcur);
          o.c = c_dd * dj + c_dr * s.dinv[k] * o.b;
        }
        return o;
      }, [&](int k, F3 v) {
        tpool[ti(g, TA_X, tj(g, k))] = v.a;
        if (!last) {
          tpool[ti(g, TA_R, tj(g, k))] = v.b;
          tpool[ti(g, dn, tj(g, k))] = v.c;
        }
      });
      dcur = dn;
    }
  }
  return false;
}

__device__ __forceinline__ bool tail_down_any(const InstDesc &D, const TailSm &m,
                                              const TailLevel &f, const TailLevel &g,
                                              bool restrict_in, bool smooth) {
  switch (tail_per(g.n)) {
    case 1: return tail_down<1>(D, m, f, g, restrict_in, smooth);
    case 2: return tail_down<2>(D, m, f, g, restrict_in, smooth);
    case 3: return tail_down<3>(D, m, f, g, restrict_in, smooth);
    default: return tail_down<4>(D, m, f, g, restrict_in, smooth);
  }
}

__device__ __forceinline__ bool tail_up_any(const InstDesc &D, const TailSm &m,
                                            const TailLevel &g, const TailLevel &c, int ca,
                                            bool in_da) {
  switch (tail_per(g.n)) {
    case 1: return tail_up<1>(D, m, g, c, ca, in_da);
    case 2: return tail_up<2>(D, m, g, c, ca, in_da);
    case 3: return tail_up<3>(D, m, g, c, ca, in_da);
    default: return tail_up<4>(D, m, g, c, ca, in_da);
  }
}

}  // namespace

// Part `part` of `parts` of an instance's pending f, w update (Algorithm 2's update of the step
// before: f += (phi/rho) w, w = v/alpha - (theta/rho) w; n % 4 == 0), run by the extra
// workgroups of a tail launch. It ignores the stop flag: a pending update comes from a step that
// completed, and whatever stopped later leaves it to be applied.
__device__ __forceinline__ void tail_update_part(const InstDesc &D, int part, int parts) {
  const double *sc = sld(D.sc);
  if (sc[SC_UPD] == 0.0) return;
  const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW], sv = (float)sc[SC_SV];
  const long long n4 = sld(D.n) / 4;
  const long long per = (n4 + parts - 1) / parts;
  const long long b = per * part, e = min(n4, b + per);
  float4 *__restrict__ f = reinterpret_cast<float4 *>(sld(D.f));
  float4 *__restrict__ w = reinterpret_cast<float4 *>(sld(D.w));
  const float4 *__restrict__ v = reinterpret_cast<const float4 *>(sld(D.v));
  // two groups per trip, every load of the trip issued before the first store
  for (long long i0 = b + threadIdx.x; i0 < e; i0 += 2 * kTailBlock) {
    const long long i1 = i0 + kTailBlock;
    const bool h1 = i1 < e;
    const long long j1 = h1 ? i1 : i0;
    float4 w0 = w[i0], f0 = f[i0];
    const float4 v0 = v[i0];
    float4 w1 = w[j1], f1 = f[j1];
    const float4 v1 = v[j1];
    f0.x += cf * w0.x; f0.y += cf * w0.y; f0.z += cf * w0.z; f0.w += cf * w0.w;
    w0.x = sv * v0.x - cw * w0.x; w0.y = sv * v0.y - cw * w0.y;
    w0.z = sv * v0.z - cw * w0.z; w0.w = sv * v0.w - cw * w0.w;
    f1.x += cf * w1.x; f1.y += cf * w1.y; f1.z += cf * w1.z; f1.w += cf * w1.w;
    w1.x = sv * v1.x - cw * w1.x; w1.y = sv * v1.y - cw * w1.y;
    w1.z = sv * v1.z - cw * w1.z; w1.w = sv * v1.w - cw * w1.w;
    f[i0] = f0;
    w[i0] = w0;
    if (h1) {
      f[i1] = f1;
      w[i1] = w1;
    }
  }
}

// Block (0, i): the tail of instance i. Blocks (1 .. gridDim.x - 1, i): the parts of instance
// i's pending f, w update (a launch with update parts).
__global__ void __launch_bounds__(kTailBlock) k_vcycle_tail_lds(InstDesc *const *descs, int t) {
  const InstDesc &D = inst(descs);
  if (blockIdx.x > 0) {
    tail_update_part(D, (int)blockIdx.x - 1, (int)gridDim.x - 1);
    return;
  }
  if (stopped_inner(D)) return;
  if (t < 0) t = sld(D.tail_lds_t);   // instances of different hierarchies in one launch
  const int Lv = sld(D.levels);
  // the Chebyshev coefficients of each step, once
  if (sld(D.smoother) != PLSQR_SMOOTH_JACOBI && (int)threadIdx.x < sld(D.cheb_degree)) {
    float c_dd, c_dr;
    cheb_coef(D, threadIdx.x, c_dd, c_dr);
    tcdd[threadIdx.x] = c_dd;
    tcdr[threadIdx.x] = c_dr;
  }
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
  TailSm m;
  m.jac = sld(D.smoother) == PLSQR_SMOOTH_JACOBI;
  m.nu = sld(D.nu_pre);
  m.m = sld(D.cheb_degree);
  m.om = sld(D.omega);
  m.ith = m.jac ? 0.f : (float)(1.0 / sld(D.cheb_theta));
  // Jacobi: the current iterate alternates between TA_X and TA_DA (bit l of in_da: level l's
  // iterate is in TA_DA)
  unsigned in_da = 0;

  // ---- down: levels t .. coarsest - 1 smoothed, each level below t restricted into --------
  for (int l = t; l < Lv; ++l) {
    const TailLevel g = tail_level(D, t, l);
    const TailLevel f = (l > t) ? tail_level(D, t, l - 1) : g;
    if (tail_down_any(D, m, f, g, l > t, l < Lv - 1)) in_da |= 1u << l;
  }

  // ---- coarsest: x = A_c^{-1} b with the FP64 inverse ---------------------------------------
  {
    // each row of the inverse split over gl lanes (the largest power of two <= min(64,
    // kTailBlock / nc)); when every row fits one pass and a lane's share of a row is at most
    // kTailAi entries, that share is loaded before b is converted, so the loads overlap it
    const int nc = sld(D.lv[Lv - 1].n);
    int gl = 1;
    while (2 * gl <= 64 && 2 * gl * nc <= kTailBlock) gl *= 2;
    const int lane = threadIdx.x % gl;
    const int rows_per_pass = kTailBlock / gl;
    const bool ai_regs = rows_per_pass >= nc && (nc + gl - 1) / gl <= kTailAi;
    const double *__restrict__ Ai = sld(D.cfac) + (long long)nc * nc * 2;
    double ai[kTailAi];
    if (ai_regs) {
      const int i = min((int)threadIdx.x / gl, nc - 1);
#pragma unroll
      for (int q = 0; q < kTailAi; ++q) ai[q] = Ai[(long long)min(lane + q * gl, nc - 1) * nc + i];
    }
    const TailLevel g = tail_level(D, t, Lv - 1);
    for (int i = threadIdx.x; i < nc; i += kTailBlock) tbs[i] = (double)tpool[ti(g, TA_B, i)];
    __syncthreads();
    for (int i0 = 0; i0 < nc; i0 += rows_per_pass) {
      const int i = i0 + (int)threadIdx.x / gl;
      double acc = 0.0;
      if (ai_regs) {
#pragma unroll
        for (int q = 0; q < kTailAi; ++q)
          if (lane + q * gl < nc) acc += ai[q] * tbs[lane + q * gl];
      } else if (i < nc) {
        for (int jj = lane; jj < nc; jj += gl) acc += Ai[(long long)jj * nc + i] * tbs[jj];
      }
      for (int o = 1; o < gl; o <<= 1) acc += __shfl_xor(acc, o, 64);
      if (i < nc && lane == 0) tpool[ti(g, TA_X, i)] = (float)acc;
    }
    __syncthreads();
  }

  // ---- up ----------------------------------------------------------------------------------
  for (int l = Lv - 2; l >= t; --l) {
    const TailLevel g = tail_level(D, t, l);
    const TailLevel c = tail_level(D, t, l + 1);
    // the coarse level's iterate: the coarsest solve writes TA_X, a smoothed level the array its
    // last sweep wrote
    const int ca = ((in_da >> (l + 1)) & 1u) ? TA_DA : TA_X;
    const bool da = tail_up_any(D, m, g, c, ca, (in_da >> l) & 1u);
    in_da = (in_da & ~(1u << l)) | ((da ? 1u : 0u) << l);
  }
  // level t's iterate back to global memory for the level above
  {
    const LevelDesc L = level_of(D, t);
    const TailLevel g = tail_level(D, t, t);
    const int a = (m.jac && ((in_da >> t) & 1u)) ? TA_DA : TA_X;
    for (int j = threadIdx.x; j < g.n; j += kTailBlock) L.x[j] = tpool[ti(g, a, j)];
  }
}

long long tail_lds_floats(const long long *cells, int nlev) {
  long long s = 0;
  for (int i = 0; i < nlev; ++i) s += (long long)TA_COUNT * cells[i];
  return s;
}

void launch_vcycle_tail_lds(hipStream_t st, InstDesc *const *d, int B, int t, int upd_parts) {
  hipLaunchKernelGGL(k_vcycle_tail_lds, dim3(1 + upd_parts, B), dim3(kTailBlock), 0, st, d, t);
}

}  // namespace plsqr
