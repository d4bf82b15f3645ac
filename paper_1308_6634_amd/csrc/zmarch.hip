// Fused multigrid level kernels: one launch runs a level's whole pre-smoothing together with
// the residual restriction ("down"), or the prolongation together with the whole
// post-smoothing ("up"), of the V-cycle that applies the priorconditioner (section 4.2).
//
// Temporal blocking by marching along z. A block owns an output tile of tx x ty columns
// (x fastest) and a chunk of zc planes. Its threads cover the tile widened by the halo the
// smoother needs (H = the number of stencil applications, at most 4: H rows on each y side,
// and on each x side H voxels, or one group of four when a thread owns four x-consecutive
// voxels). The block marches through the planes: in iteration t, stage 0 forms the first
// stencil input at plane t, and stage s (1..H) applies the level stencil at plane t - s, so
// each stage runs one plane behind the previous one. A stage takes its z-neighbours from the
// thread's own registers (the values the previous stage produced at the planes on either side)
// and its x/y-neighbours from the LDS copy of the previous stage's plane written in the
// preceding iteration; one barrier per iteration orders the LDS. Columns near the widened
// tile's edge compute values that are never used (their neighbours are missing), and the loss
// shrinks the valid region by one column per stage, which the halo absorbs.
//
// A thread owns V = 4 x-consecutive voxels (16-byte loads; for levels that keep the chip busy,
// where the instruction count per voxel decides) or V = 1 voxel (four times as many threads
// and a quarter of the instructions per iteration, for the small levels, where one block's
// march along z decides).
//
// The inputs of a plane (right-hand side, face weights, the level's stored 1/diag) are loaded
// once, ahead of their first use, and handed down the stages in registers.
//
// Every voxel's arithmetic is that of the one-pass kernels (smooth_vec.hip): the same formulas
// with the terms in the same order, so the fused and the per-sweep V-cycles give the same
// values up to the sign of a zero sum; only the alpha partial sums are grouped differently.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

// threads per block: a four-voxel thread carries about four times the registers; a one-voxel
// block covers at most (32 + 2H) x (8 + 2H) columns, 640 at H = 4, which leaves a one-voxel
// thread about 168 registers for its two planes of loads in flight
constexpr int kZmMaxThreads = 640;
__host__ __device__ constexpr int zm_max_threads(int V) { return V == 4 ? 512 : 640; }

// Planes of loads a thread keeps in flight (see k_zm), from the register counts of the variants:
// two where the thread holds two slots without spilling (one-voxel threads but for the coarse
// degree-4 Chebyshev smoothing, and the level-0 four-voxel variants below), else one.
__host__ __device__ constexpr int zm_prefetch(int kind, int H, bool L0, int V) {
  return V == 1 ? ((!L0 && (kind == ZM_CHEB_DOWN || kind == ZM_CHEB_UP) && H == 4) ? 1 : 2)
         : !L0  ? 1
         : (kind == ZM_JAC_DOWN) ? (H <= 3 ? 2 : 1)
         : (kind == ZM_JAC_UP)   ? (H <= 3 ? 2 : 1)
         : (kind == ZM_CHEB_DOWN) ? (H <= 3 ? 2 : 1)
                                  : (H <= 2 ? 2 : 1);
}

template <int V>
struct Vec {
  float v[V];
};

template <int V>
__device__ __forceinline__ Vec<V> ldv(const float *p) {
  Vec<V> r;
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    r.v[0] = t.x;
    r.v[1] = t.y;
    r.v[2] = t.z;
    r.v[3] = t.w;
  } else {
    r.v[0] = *p;
  }
  return r;
}
template <int V>
__device__ __forceinline__ void stv(float *p, const Vec<V> &a) {
  if constexpr (V == 4) *reinterpret_cast<float4 *>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
  else *p = a.v[0];
}
// LDS cell of one thread: a float4 for V = 4, a float for V = 1
template <int V>
using LdsCell = typename std::conditional<V == 4, float4, float>::type;
template <int V>
__device__ __forceinline__ LdsCell<V> to_cell(const Vec<V> &a) {
  if constexpr (V == 4) return make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
  else return a.v[0];
}
template <int V>
__device__ __forceinline__ Vec<V> from_cell(const LdsCell<V> &c) {
  Vec<V> r;
  if constexpr (V == 4) {
    r.v[0] = c.x;
    r.v[1] = c.y;
    r.v[2] = c.z;
    r.v[3] = c.w;
  } else {
    r.v[0] = c;
  }
  return r;
}
template <int V>
__device__ __forceinline__ float first_of(const LdsCell<V> &c) {
  if constexpr (V == 4) return c.x;
  else return c;
}
template <int V>
__device__ __forceinline__ float last_of(const LdsCell<V> &c) {
  if constexpr (V == 4) return c.w;
  else return c;
}

// f(std::integral_constant<int, I>{}) for I = 0 .. N - 1, unrolled.
template <int... I, class F>
__device__ __forceinline__ void static_for_seq(std::integer_sequence<int, I...>, F &&f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_seq(std::make_integer_sequence<int, N>{}, f);
}

// One thread's inputs at one plane, loaded once (two iterations ahead of their first use) and
// handed down the stages in registers: the right-hand side, the face weights to the +x/+y/+z
// neighbours (level 0: all three are kappa of the cell), the weight from the -x neighbour of
// the first voxel and the weights from the -y neighbours (as loaded, where a face leaves the
// grid, an unrelated weight: masked to zero when the plane enters), and 1/diag (the level's
// stored diagonal, formed once per outer step in the same order as the stencil's terms). The
// weights from the -z neighbours are the +z weights of the plane below, the next entry of the
// same register line. Nothing is computed from the loaded values until the plane enters, so
// the loads stay in flight until then.
template <bool L0, int V>
struct PlaneData {
  Vec<V> b, wx, wy, wz, wym, dinv;
  float wxl;
};
template <int V>
struct PlaneData<true, V> {
  Vec<V> b, k, wym, dinv;
  float wxl;
};

struct ZmCtx {
  LevelDesc L;
  int nx, ny, nz;
  long long sy, sz;
  int gx, gy;          // this thread's first voxel (global x) and row
  float eps;
};

// Loads of plane p (clamped into the grid, and for threads outside the grid from index 0, so
// that every address is valid and no load waits on a branch); values of planes outside the
// grid are never used.
template <bool L0, int V>
__device__ __forceinline__ PlaneData<L0, V> load_plane(const ZmCtx &c, const float *__restrict__ kap,
                                                       bool in, long long col, int p) {
  const int pc = min(max(p, 0), c.nz - 1);
  const long long j = in ? col + c.sz * pc : 0;
  const bool hl = in && c.gx > 0, hy = in && c.gy > 0;   // the -x / -y faces exist
  const long long jl = hl ? j - 1 : j;
  const long long jy = hy ? j - c.sy : j;
  PlaneData<L0, V> d;
  d.dinv = ldv<V>(c.L.dinv + j);
  d.b = ldv<V>(c.L.b + j);
  const float *wxs = L0 ? kap : c.L.wx;
  const float *wys = L0 ? kap : c.L.wy;
  d.wxl = wxs[jl];
  d.wym = ldv<V>(wys + jy);
  if constexpr (L0) {
    d.k = ldv<V>(kap + j);
  } else {
    d.wx = ldv<V>(c.L.wx + j);
    d.wy = ldv<V>(c.L.wy + j);
    if (c.nz > 1) d.wz = ldv<V>(c.L.wz + j);
    else d.wz = Vec<V>{};
  }
  return d;
}

// A register move the compiler cannot fold away. In the paired form (below) a prefetch slot is
// read through it when its plane is used: the slot's registers are then dead, the next loads
// into the slot can reuse them, and the loop carries the slot without copying registers whose
// loads are in flight (such a copy waits for every outstanding load).
__device__ __forceinline__ float vmove(float x) {
  float y;
  asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}
template <int V>
__device__ __forceinline__ Vec<V> vmove(const Vec<V> &a) {
  Vec<V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) r.v[e] = vmove(a.v[e]);
  return r;
}
template <bool L0, int V>
__device__ __forceinline__ PlaneData<L0, V> take_plane(const PlaneData<L0, V> &p) {
  PlaneData<L0, V> d;
  d.b = vmove<V>(p.b);
  if constexpr (L0) {
    d.k = vmove<V>(p.k);
  } else {
    d.wx = vmove<V>(p.wx);
    d.wy = vmove<V>(p.wy);
    d.wz = vmove<V>(p.wz);
  }
  d.wym = vmove<V>(p.wym);
  d.wxl = vmove(p.wxl);
  d.dinv = vmove<V>(p.dinv);
  return d;
}

// A plane entering the stages: the weights from the -x neighbour of the first voxel and from the
// -y neighbours masked to zero where those faces leave the grid (the stencil adds their terms
// unconditionally).
template <bool L0, int V>
__device__ __forceinline__ void mask_plane(const ZmCtx &c, PlaneData<L0, V> &d) {
  const bool hxl = c.gx > 0, hym = c.gy > 0;
  d.wxl = hxl ? d.wxl : 0.f;
#pragma unroll
  for (int e = 0; e < V; ++e) d.wym.v[e] = hym ? d.wym.v[e] : 0.f;
}

// (A_l x) at plane p, with the neighbour values given: xl/xr the x-neighbours of the first and
// last voxel, yp/ym/zp/zm the neighbouring rows and planes. The faces are added in the order of
// stencil4. Faces that leave the grid are skipped; for the -x face of the grid's first voxel and
// the -y faces the term is added anyway with the weight masked to zero (mask_plane), which
// changes nothing but the sign of a zero sum. The z faces depend only on the plane, so they are
// tested once (a uniform branch).
template <bool L0, int V>
__device__ __forceinline__ Vec<V> apply_stencil(const ZmCtx &c, const PlaneData<L0, V> &d,
                                                const PlaneData<L0, V> &below, int p,
                                                const Vec<V> &xc, float xl, float xr,
                                                const Vec<V> &yp, const Vec<V> &ym,
                                                const Vec<V> &zp, const Vec<V> &zm) {
  const bool hyp = c.gy + 1 < c.ny, hzp = p + 1 < c.nz, hzm = p > 0;
  const bool hxr = c.gx + V < c.nx;            // +x face of the last voxel
  Vec<V> acc;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const float xj = xc.v[e];
    float a = c.eps * xj;
    const float xnext = (e < V - 1) ? xc.v[e < V - 1 ? e + 1 : 0] : xr;
    const float xprev = (e > 0) ? xc.v[e > 0 ? e - 1 : 0] : xl;
    float wxp, wm, wyp;
    if constexpr (L0) {
      wxp = wyp = d.k.v[e];
      wm = (e > 0) ? d.k.v[e > 0 ? e - 1 : 0] : d.wxl;
    } else {
      wxp = d.wx.v[e];
      wyp = d.wy.v[e];
      wm = (e > 0) ? d.wx.v[e > 0 ? e - 1 : 0] : d.wxl;
    }
    if (e < V - 1 || hxr) a += wxp * (xj - xnext);
    a += wm * (xj - xprev);                     // zero weight at the grid's -x edge
    if (hyp) a += wyp * (xj - yp.v[e]);
    a += d.wym.v[e] * (xj - ym.v[e]);           // zero weight at the grid's -y edge
    acc.v[e] = a;
  }
  if (L0 || c.nz > 1) {
    if (hzp) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        float w;
        if constexpr (L0) w = d.k.v[e];
        else w = d.wz.v[e];
        acc.v[e] += w * (xc.v[e] - zp.v[e]);
      }
    }
    if (hzm) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        float w;
        if constexpr (L0) w = below.k.v[e];
        else w = below.wz.v[e];
        acc.v[e] += w * (xc.v[e] - zm.v[e]);
      }
    }
  }
  return acc;
}

__device__ __forceinline__ double block_sum_any(double v) {
  __shared__ double red[kZmMaxThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += red[i];
  return r;
}

// threads of x halo on each side: one group of four, or H single voxels
__host__ __device__ constexpr int halo_units(int V, int H) { return V == 4 ? 1 : H; }

}  // namespace

// KIND: ZM_JAC_DOWN, ZM_JAC_UP (damped Jacobi, H = nu sweeps), ZM_CHEB_DOWN, ZM_CHEB_UP
// (one Chebyshev polynomial of degree H per side); L0: level 0 (face weights are kappa);
// V: voxels per thread. Down: b = level l's right-hand side -> pre-smoothed iterate into L.t,
// restricted residual into b of level l + 1. Up: L.t and the coarse correction x of level
// l + 1 -> post-smoothed iterate into L.x (on level 0 that is v, and with want_dot the block's
// part of v.p).
template <int KIND, int H, bool L0, int V>
__global__ void __launch_bounds__(zm_max_threads(V)) k_zm(InstDesc *const *descs, int l, int tx,
                                                     int ty, int zc, int want_dot, Rag rg) {
  constexpr bool DOWN = (KIND == ZM_JAC_DOWN || KIND == ZM_CHEB_DOWN);
  constexpr bool CHEB = (KIND == ZM_CHEB_DOWN || KIND == ZM_CHEB_UP);
  constexpr int HX = halo_units(V, H);
  using Cell = LdsCell<V>;
  extern __shared__ float4 zsm4[];
  Cell *zsm = reinterpret_cast<Cell *>(zsm4);
  const Blk blk = locate(rg);
  if (blk.i < 0) return;
  const InstDesc &D = *descs[blk.i];
  if (stopped_inner(D)) return;
  if (tx == 0) {   // a ragged launch: this instance's own tile of level l
    tx = sld(D.zmp[l].tx);
    ty = sld(D.zmp[l].ty);
    zc = sld(D.zmp[l].zc);
  }
  ZmCtx c;
  c.L = level_of(D, l);
  const LevelDesc Cl = level_of(D, l + 1);
  c.nx = c.L.nx;
  c.ny = c.L.ny;
  c.nz = c.L.nz;
  c.sy = c.nx;
  c.sz = (long long)c.nx * c.ny;
  c.eps = (float)c.L.eps;
  const float *__restrict__ kap = L0 ? sld(D.kappa) : nullptr;
  const int ntx = (c.nx + tx - 1) / tx, nty = (c.ny + ty - 1) / ty, ntz = (c.nz + zc - 1) / zc;
  const long long b = xcd_tile_of(blk);
  if (b >= (long long)ntx * nty * ntz) {   // past this instance's tiles (a larger batch member)
    if (want_dot && threadIdx.x == 0) sld(D.part)[blk.bx] = 0.0;
    return;
  }
  const int bx = (int)(b % ntx), by = (int)((b / ntx) % nty), bz = (int)(b / ((long long)ntx * nty));
  const int x0 = bx * tx, y0 = by * ty, z0 = bz * zc;
  const int exq = tx / V + 2 * HX, ey = ty + 2 * H;
  const int plane = exq * ey;               // LDS cells per plane
  const int q = (int)threadIdx.x % exq, row = (int)threadIdx.x / exq;
  c.gx = x0 - HX * V + V * q;
  c.gy = y0 - H + row;
  const bool live = row < ey;
  const bool in = live && c.gx >= 0 && c.gx < c.nx && c.gy >= 0 && c.gy < c.ny;
  const bool out = in && q >= HX && q < HX + tx / V && row >= H && row < H + ty;
  const int qm = q > 0 ? q - 1 : 0, qp = q + 1 < exq ? q + 1 : exq - 1;
  const int rm = row > 0 ? row - 1 : 0, rp = row + 1 < ey ? row + 1 : ey - 1;
  const int lrow = live ? row : 0;
  const long long col = (long long)c.gx + c.sy * c.gy;   // global index at plane 0
  auto zb = [&](int par, int s) { return zsm + (par * H + s) * plane; };
  auto rbuf = [&](int par) { return zsm + (2 * H + par) * plane; };

  const float om = sld(D.omega);
  const float ith = CHEB ? (float)(1.0 / sld(D.cheb_theta)) : 0.f;
  float cdd[H], cdr[H];   // Chebyshev step coefficients (the recurrence of the one-pass kernels)
  if (CHEB) {
    const double sigma = sld(D.cheb_sigma), delta = sld(D.cheb_delta);
    double rho = 1.0 / sigma;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      cdd[k] = (float)(rn * rho);
      cdr[k] = (float)(2.0 * rn / delta);
      rho = rn;
    }
  }
  const float *__restrict__ xpre = c.L.t;    // up: the pre-smoothed iterate
  const float *__restrict__ ecrs = Cl.x;     // up: coarse correction
  const int czf = (c.nz > 1) ? 2 : 1;        // fine planes per coarse plane
  const int czs = czf - 1;                   // its shift: coarse plane = fine plane >> czs
  // the coarse cell of this thread's column (x, y halved) in coarse plane 0, and the coarse
  // plane size: a coarse index is cbase + csz * plane (32-bit: levels hold < 2^31 cells)
  const long long cbase = (long long)(c.gx >> 1) + (long long)Cl.nx * (c.gy >> 1);
  const int csz = Cl.nx * Cl.ny;
  const int zend = min(c.nz, z0 + zc);      // output planes [z0, zend)
  const int t0 = max(0, z0 - H);
  const int t1 = zend - 1 + H + (DOWN ? 1 : 0);
  const int phi0 = min(c.nz - 1, zend - 1 + H);   // last plane stage 0 works on

  // The inputs of the planes the stages read (t .. t - H - 1: stage s works on plane t - s and
  // takes its -z weights from the plane below) and of the PF planes whose loads are in flight
  // (PF = 2, or one where two would not fit the registers of a four-voxel thread without
  // spilling: a spill reload in the loop would wait for the loads issued before it). Three forms:
  // * ring (four voxels per thread, PF = 2): R slots, plane t0 + i in slot i mod R, the plane
  //   below the first in slot R - 1, and the march unrolled R times (the iteration's offset
  //   U = (t - t0) mod R is a compile-time constant), so a plane keeps its registers from its
  //   loads to its last use and nothing rotates;
  // * pair (one voxel per thread, PF = 2; their marches are short, where the ring's longer code
  //   cost more than it saved): the planes shift down a register line (pd) each iteration, two
  //   prefetch slots taken alternately by iterations run in pairs;
  // * single (PF = 1): the same line behind one prefetch slot.
  using PD = PlaneData<L0, V>;
  constexpr int PF = zm_prefetch(KIND, H, L0, V);
  constexpr int FORM = (PF == 2) ? (V == 4 ? 0 : 1) : 2;   // ring, pair, single
  constexpr int R = (FORM == 0) ? H + 2 + PF : 1;
  struct UpData {     // up: the pre-smoothed iterate and the coarse correction of a plane
    Vec<V> x;
    float e0, e1;
  };
  PD ring[R];
  UpData upr[R];
  PD pd[H + 2];       // pair and single forms: the planes t .. t - H - 1
  PD pfs[2];          // their prefetch slots
  UpData ups[2];
  Vec<V> cur_x = {};                   // up: pre-smoothed iterate of the current plane
  float cur_e0 = 0.f, cur_e1 = 0.f;
  auto up_loads = [&](int p, UpData &u) {
    const int pc = min(max(p, 0), c.nz - 1);
    const long long j = in ? col + c.sz * pc : 0;
    const long long pj = in ? cbase + csz * (pc >> czs) : 0;
    u.x = ldv<V>(xpre + j);
    u.e0 = ecrs[pj];
    u.e1 = (V == 4) ? ecrs[pj + 1] : 0.f;
  };
  {
    // the plane below the first one (its weights are the -z weights of the stencil at the
    // first plane); clamped to plane 0, and then unused, when t0 == 0. Loaded first, then the
    // first PF planes. The other slots are written before any stage reads them.
    const PD below = load_plane<L0, V>(c, kap, in, col, t0 - 1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      ring[k] = below;
      upr[k] = UpData{};
    }
#pragma unroll
    for (int k = 0; k < H + 2; ++k) pd[k] = below;
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const PD pl = load_plane<L0, V>(c, kap, in, col, min(t0 + k, phi0));
    UpData ul{};
    if (!DOWN) up_loads(min(t0 + k, phi0), ul);
    if constexpr (FORM == 0) {
      ring[k] = pl;
      upr[k] = ul;
    } else {
      pfs[k] = pl;
      ups[k] = ul;
    }
  }

  // z-lines of the stencil inputs: zcv[s], zmv[s] = stage-s input at the plane stage s works on
  // and the one below; znv[s] = what stage s-1 produced in this iteration (the plane above)
  Vec<V> zcv[H + 1], zmv[H + 1], znv[H + 1];
  Vec<V> sx[H + 1], sr[H + 1];      // pointwise state passed from stage s-1 to stage s
  Vec<V> nsx[H + 1], nsr[H + 1];
#pragma unroll
  for (int s = 0; s <= H; ++s) {
    zcv[s] = Vec<V>{};
    zmv[s] = Vec<V>{};
    znv[s] = Vec<V>{};
    sx[s] = Vec<V>{};
    sr[s] = Vec<V>{};
    nsx[s] = Vec<V>{};
    nsr[s] = Vec<V>{};
  }
  Vec<V> rlast = {};          // down: the residual of the plane stage H finished last iteration
  float racc0 = 0.f, racc1 = 0.f;
  double dot = 0.0;

  // offset: U (the ring form) or the prefetch slot (the others), as a compile-time constant
  auto iteration = [&](auto offset, const int t) __attribute__((always_inline)) {
    constexpr int U = decltype(offset)::value;
    // the inputs of plane t - s
    auto plane = [&](int s) -> PD & {
      if constexpr (FORM == 0) return ring[(U + R - s) % R];
      else return pd[s];
    };
    const int cur = t & 1, prev = cur ^ 1;
    // the entering plane, masked; then the loads of the plane PF ahead (unconditional, the plane
    // is clamped, so that no branch join makes them complete early)
    const int pnext = min(t + PF, phi0);
    if constexpr (FORM == 0) {
      mask_plane<L0, V>(c, ring[U]);
      if (!DOWN) {
        cur_x = upr[U].x;
        cur_e0 = upr[U].e0;
        cur_e1 = upr[U].e1;
      }
      ring[(U + PF) % R] = load_plane<L0, V>(c, kap, in, col, pnext);
      if (!DOWN) up_loads(pnext, upr[(U + PF) % R]);
    } else {
#pragma unroll
      for (int s = H + 1; s > 0; --s) pd[s] = pd[s - 1];
      if constexpr (FORM == 1) {
        pd[0] = take_plane<L0, V>(pfs[U]);
        if (!DOWN) {
          cur_x = vmove<V>(ups[U].x);
          cur_e0 = vmove(ups[U].e0);
          if (V == 4) cur_e1 = vmove(ups[U].e1);
        }
      } else {
        pd[0] = pfs[U];
        if (!DOWN) {
          cur_x = ups[U].x;
          cur_e0 = ups[U].e0;
          cur_e1 = ups[U].e1;
        }
      }
      mask_plane<L0, V>(c, pd[0]);
      pfs[U] = load_plane<L0, V>(c, kap, in, col, pnext);
      if (!DOWN) up_loads(pnext, ups[U]);
    }
    // ---- down: restriction of the residual finished in the previous iteration ------------
    // (the children of a coarse cell, summed in the order of the one-pass restriction: for
    // each of its fine planes, the row pair in y, each row's pair in x)
    if (DOWN) {
      const int pr = t - 1 - H;
      const bool even_x = (V == 4) || ((c.gx & 1) == 0);
      if (pr >= z0 && pr < zend && out && ((row - H) & 1) == 0 && even_x) {
        const Cell *rb = rbuf(prev);
        if constexpr (V == 4) {
          const float4 nb = rb[rp * exq + q];
          racc0 += rlast.v[0];
          racc0 += rlast.v[1];
          racc1 += rlast.v[2];
          racc1 += rlast.v[3];
          racc0 += nb.x;
          racc0 += nb.y;
          racc1 += nb.z;
          racc1 += nb.w;
        } else {
          racc0 += rlast.v[0];
          racc0 += rb[lrow * exq + qp];
          racc0 += rb[rp * exq + q];
          racc0 += rb[rp * exq + qp];
        }
        if (czf == 1 || (pr & 1)) {
          const long long J = cbase + csz * (pr >> czs);   // pr >= z0 >= 0
          if constexpr (V == 4) *reinterpret_cast<float2 *>(Cl.b + J) = make_float2(racc0, racc1);
          else Cl.b[J] = racc0;
          racc0 = 0.f;
          racc1 = 0.f;
        }
      }
    }
    // ---- stage 0 at plane t: the first stencil input ------------------------------------
    {
      Vec<V> z1 = {};
      const int p = t;
      if (in && p <= phi0) {
        if (DOWN) {
          const Vec<V> &dv = plane(0).dinv;
#pragma unroll
          for (int e = 0; e < V; ++e) z1.v[e] = (CHEB ? ith : om) * dv.v[e] * plane(0).b.v[e];
        } else {
          // x' = x + P e: voxel pairs along x share one coarse parent
          z1 = cur_x;
#pragma unroll
          for (int e = 0; e < V; ++e) z1.v[e] += (e < 2) ? cur_e0 : cur_e1;
        }
        nsx[1] = z1;                                 // x after the first sweep / step, or x'
      }
      znv[1] = z1;
      if (live) zb(cur, 0)[lrow * exq + q] = to_cell<V>(z1);
    }
    // ---- stages 1..H at planes t-1 .. t-H ---------------------------------------------------
#pragma unroll
    for (int s = 1; s <= H; ++s) {
      const int p = t - s;
      const int plo = max(0, z0 - (H - s)), phi = min(c.nz - 1, zend - 1 + (H - s));
      const bool act = in && p >= plo && p <= phi;
      Vec<V> znext = {};
      if (act) {
        const long long j = col + c.sz * p;
        const Cell *zp_ = zb(prev, s - 1);
        const Vec<V> ym = from_cell<V>(zp_[rm * exq + q]), yp = from_cell<V>(zp_[rp * exq + q]);
        const float xl = last_of<V>(zp_[lrow * exq + qm]), xr = first_of<V>(zp_[lrow * exq + qp]);
        const PD &d = plane(s);
        const Vec<V> xc = zcv[s];
        const Vec<V> ax = apply_stencil<L0, V>(c, d, plane(s + 1), p, xc, xl, xr, yp, ym, znv[s],
                                               zmv[s]);
        const Vec<V> &dv = d.dinv;
        const Vec<V> &bb = d.b;
        if (KIND == ZM_JAC_DOWN || KIND == ZM_JAC_UP) {
          const bool last = (s == H);
          if (DOWN && last) {
            // residual of the pre-smoothed iterate (xc): restricted next iteration
            Vec<V> r;
#pragma unroll
            for (int e = 0; e < V; ++e) r.v[e] = bb.v[e] - ax.v[e];
            rlast = r;
            rbuf(cur)[lrow * exq + q] = to_cell<V>(r);
            if (out) stv<V>(c.L.t + j, xc);
          } else {
            Vec<V> xn;
#pragma unroll
            for (int e = 0; e < V; ++e) xn.v[e] = xc.v[e] + om * dv.v[e] * (bb.v[e] - ax.v[e]);
            if (last) {   // up: the post-smoothed iterate
              if (out) {
                stv<V>(c.L.x + j, xn);
                if (want_dot) {
                  double dq = 0.0;
#pragma unroll
                  for (int e = 0; e < V; ++e) dq += (double)xn.v[e] * (double)bb.v[e];
                  dot += dq;
                }
              }
            } else {
              znext = xn;
            }
          }
        } else if (KIND == ZM_CHEB_DOWN) {
          // stage s applies the stencil to d_{s-1}; x already holds d_0 + .. + d_{s-2}
          Vec<V> r, xn;
          if (s == 1) {
#pragma unroll
            for (int e = 0; e < V; ++e) r.v[e] = bb.v[e] - ax.v[e];
            xn = sx[1];                              // x = d_0
          } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              xn.v[e] = sx[s].v[e] + xc.v[e];
              r.v[e] = sr[s].v[e] - ax.v[e];
            }
          }
          if (s < H) {
#pragma unroll
            for (int e = 0; e < V; ++e) znext.v[e] = cdd[s - 1] * xc.v[e] + cdr[s - 1] * dv.v[e] * r.v[e];
            nsx[s + 1] = xn;
            nsr[s + 1] = r;
          } else {
            rlast = r;
            rbuf(cur)[lrow * exq + q] = to_cell<V>(r);
            if (out) stv<V>(c.L.t + j, xn);
          }
        } else {   // ZM_CHEB_UP
          // stage 1: r = b - A x', d_0 = D^{-1} r / theta; stage s >= 2: x += d_{s-2},
          // r -= A d_{s-2}, d_{s-1}; after the last stage x += d_{H-1} is the result
          Vec<V> r, xn, dn;
          if (s == 1) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              r.v[e] = bb.v[e] - ax.v[e];
              dn.v[e] = ith * dv.v[e] * r.v[e];
            }
            xn = sx[1];                              // x' (the first step adds d_0 to it)
          } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              xn.v[e] = sx[s].v[e] + xc.v[e];
              r.v[e] = sr[s].v[e] - ax.v[e];
              dn.v[e] = cdd[s - 2] * xc.v[e] + cdr[s - 2] * dv.v[e] * r.v[e];
            }
          }
          if (s < H) {
            znext = dn;
            nsx[s + 1] = xn;
            nsr[s + 1] = r;
          } else {
            Vec<V> xf;
#pragma unroll
            for (int e = 0; e < V; ++e) xf.v[e] = xn.v[e] + dn.v[e];
            if (out) {
              stv<V>(c.L.x + j, xf);
              if (want_dot) {
                double dq = 0.0;
#pragma unroll
                for (int e = 0; e < V; ++e) dq += (double)xf.v[e] * (double)bb.v[e];
                dot += dq;
              }
            }
          }
        }
      }
      if (s < H) {
        znv[s + 1] = znext;
        if (live) zb(cur, s)[lrow * exq + q] = to_cell<V>(znext);
      }
    }
    // ---- shift the z-lines and the passed state by one plane --------------------------------
#pragma unroll
    for (int s = 1; s <= H; ++s) {
      zmv[s] = zcv[s];
      zcv[s] = znv[s];
      sx[s] = nsx[s];
      sr[s] = nsr[s];
    }
    __syncthreads();
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  if constexpr (FORM == 0) {
    // whole trips of R iterations, then the remaining ones after the loop: every path back to
    // the loop head has issued the loads of all R iterations in order, so the head waits only
    // for the slot it takes
    int t = t0;
    for (; t + R - 1 <= t1; t += R)
      static_for<R>([&](auto k) { iteration(k, t + decltype(k)::value); });
    static_for<R - 1>([&](auto k) {
      if (t + decltype(k)::value <= t1) iteration(k, t + decltype(k)::value);
    });
  } else if constexpr (FORM == 1) {
    // pairs of iterations (slot 0, then slot 1), then an odd last one after the loop: every
    // path back to the loop head has issued slot 1's loads after slot 0's
    int t = t0;
    for (; t + 1 <= t1; t += 2) {
      iteration(I0{}, t);
      iteration(I1{}, t + 1);
    }
    if (t <= t1) iteration(I0{}, t);
  } else {
    for (int t = t0; t <= t1; ++t) iteration(I0{}, t);
  }
  if (!DOWN && want_dot) {
    const double s = block_sum_any(dot);
    if (threadIdx.x == 0) sld(D.part)[blk.bx] = s;
  }
}

// ------------------------------------------------------------------------------------
// launcher
// ------------------------------------------------------------------------------------
namespace {
template <int KIND, bool L0, int V>
void zm_dispatch(int H, dim3 g, dim3 blk, size_t smem, hipStream_t st, InstDesc *const *d, int l,
                 int tx, int ty, int zc, int want_dot, const Rag &rg) {
  switch (H) {
    case 1: hipLaunchKernelGGL((k_zm<KIND, 1, L0, V>), g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg); break;
    case 2: hipLaunchKernelGGL((k_zm<KIND, 2, L0, V>), g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg); break;
    case 3: hipLaunchKernelGGL((k_zm<KIND, 3, L0, V>), g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg); break;
    default: hipLaunchKernelGGL((k_zm<KIND, 4, L0, V>), g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg); break;
  }
}
template <int KIND>
void zm_dispatch_level(int H, int V, dim3 g, dim3 blk, size_t smem, hipStream_t st,
                       InstDesc *const *d, int l, int tx, int ty, int zc, int want_dot,
                       const Rag &rg) {
  if (V == 4) {
    if (l == 0) zm_dispatch<KIND, true, 4>(H, g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg);
    else zm_dispatch<KIND, false, 4>(H, g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg);
  } else {
    if (l == 0) zm_dispatch<KIND, true, 1>(H, g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg);
    else zm_dispatch<KIND, false, 1>(H, g, blk, smem, st, d, l, tx, ty, zc, want_dot, rg);
  }
}
template <class... A>
void zm_dispatch_kind(int kind, A... a) {
  switch (kind) {
    case ZM_JAC_DOWN: zm_dispatch_level<ZM_JAC_DOWN>(a...); break;
    case ZM_JAC_UP: zm_dispatch_level<ZM_JAC_UP>(a...); break;
    case ZM_CHEB_DOWN: zm_dispatch_level<ZM_CHEB_DOWN>(a...); break;
    default: zm_dispatch_level<ZM_CHEB_UP>(a...); break;
  }
}

int zm_exq(const ZmShape &s, int H) { return s.tx / s.v + 2 * halo_units(s.v, H); }
}  // namespace

int zm_threads(const ZmShape &s, int H) { return zm_exq(s, H) * (s.ty + 2 * H); }

size_t zm_lds_bytes(int H, const ZmShape &s, bool down) {
  const size_t cell = s.v == 4 ? sizeof(float4) : sizeof(float);
  return (size_t)(2 * H + (down ? 2 : 0)) * zm_exq(s, H) * (s.ty + 2 * H) * cell;
}

long long zm_tiles(int nx, int ny, int nz, const ZmShape &s) {
  return (long long)((nx + s.tx - 1) / s.tx) * ((ny + s.ty - 1) / s.ty) * ((nz + s.zc - 1) / s.zc);
}

ZmShape zm_shape(int nx, int ny, int nz, int H, int ty_knob, int zc_knob, int v_knob) {
  ZmShape s;
  // four voxels per thread on levels of a million cells and more (there the instruction count
  // per voxel decides), one voxel per thread below (there one block's march decides)
  s.v = v_knob ? v_knob : ((long long)nx * ny * nz >= (1LL << 20) && nx % 4 == 0 ? 4 : 1);
  if (s.v == 4) {
    s.tx = nx < 64 ? nx : 64;
    s.ty = ty_knob > 0 ? ty_knob : 16;
  } else {
    s.tx = nx < 32 ? nx : 32;
    s.ty = ty_knob > 0 ? ty_knob : 8;
  }
  if (s.ty > ny) s.ty = ny;
  s.ty &= ~1;
  if (s.ty < 2) s.ty = 2;
  // at most zm_max_threads threads and 64 KB of LDS
  while ((zm_threads(s, H) > zm_max_threads(s.v) || zm_lds_bytes(H, s, true) > 65536) && s.ty > 2)
    s.ty -= 2;
  const long long xy = (long long)((nx + s.tx - 1) / s.tx) * ((ny + s.ty - 1) / s.ty);
  if (zc_knob > 0) {
    s.zc = zc_knob;
  } else {
    // planes per block: the most of 16, 8, 4 that still gives the instance 256 blocks (a block's
    // march takes zc + 2H iterations, so small levels take short chunks), else 2. The tile
    // depends on the instance's own grid only (never on its batch), so the partial sums of
    // v.p, hence the result, are the same alone and in any batch.
    s.zc = 2;
    for (int z = 16; z >= 4; z /= 2)
      if (xy * ((nz + z - 1) / z) >= 256) {
        s.zc = z;
        break;
      }
  }
  if (s.zc > nz) s.zc = nz;
  if (nz > 1) s.zc = (s.zc + 1) & ~1;   // coarse planes never straddle two blocks
  if (s.zc < 1) s.zc = 1;
  return s;
}

bool zm_fits(int nx, int H, const ZmShape &s) {
  return (s.v == 1 || s.v == 4) && nx % s.v == 0 && nx % 2 == 0 && H >= 1 && H <= 4 &&
         s.tx % s.v == 0 && s.tx % 2 == 0 && s.tx >= s.v && s.ty >= 2 && s.zc >= 1 &&
         zm_threads(s, H) <= zm_max_threads(s.v) && zm_lds_bytes(H, s, true) <= 65536;
}

int launch_zm(hipStream_t st, InstDesc *const *d, int B, int kind, int H, int l, int nx, int ny,
              int nz, const ZmShape &s, int want_dot) {
  const unsigned threads = (unsigned)((zm_threads(s, H) + 63) / 64 * 64);
  const unsigned tiles = (unsigned)zm_tiles(nx, ny, nz, s);
  const bool down = (kind == ZM_JAC_DOWN || kind == ZM_CHEB_DOWN);
  const size_t smem = zm_lds_bytes(H, s, down);
  zm_dispatch_kind(kind, H, s.v, dim3(tiles, B), dim3(threads), smem, st, d, l, s.tx, s.ty, s.zc,
                   want_dot, kNoRag);
  return (int)tiles;
}

void launch_zm_ragged(hipStream_t st, InstDesc *const *d, int kind, int H, int l, int v,
                      int threads, size_t lds, const Rag &rg, int want_dot) {
  const unsigned blocks = (unsigned)(rg.first[rg.n - 1] + rg.count[rg.n - 1]);
  const unsigned th = (unsigned)((threads + 63) / 64 * 64);
  zm_dispatch_kind(kind, H, v, dim3(blocks, 1), dim3(th), lds, st, d, l, 0, 0, 0, want_dot, rg);
}

}  // namespace plsqr
