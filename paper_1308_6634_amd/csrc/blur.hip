// Separable Gaussian blur, the structured forward operator A of the test problems (and its
// adjoint, the same passes with reversed taps): one 1D correlation pass per axis with zero
// values outside the grid, y[x] = sum_k w[k] src[x + k - r]. The last pass applies the Krylov
// epilogue of the bidiagonalization (section 3.2, Algorithm 2). Every pass reads and writes
// one vector, so the passes are HBM-bound; each thread loads its whole input window into
// registers at once (16-byte groups along x, one coalesced row segment per wave along y and
// z), halo re-reads coming from L1/L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "finalize.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

// The product epilogues for four consecutive voxels j..j+3 (same arithmetic per voxel as
// epilogue()); u, p and out are workspace vectors (256-byte aligned), g is read per voxel.
__device__ __forceinline__ void epilogue4(const InstDesc &D, int epi, long long j, const V4 &y,
                                          float *out, double &dot) {
  const double *sc = sld(D.sc);
  switch (epi) {
    case EPI_FWD: {
      float *du = sld(D.u);
      const float c1 = (float)sc[SC_SV], c2 = (float)(sc[SC_ALPHA] * sc[SC_SU]);
      const V4 u = ld4(du + j);
      V4 un;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        un.v[e] = c1 * y.v[e] - c2 * u.v[e];
        dot += (double)un.v[e] * (double)un.v[e];
      }
      st4(du + j, un);
      break;
    }
    case EPI_ADJ: {
      const float c1 = (float)sc[SC_SU], c2 = (float)(sc[SC_BETA] * sc[SC_SV]);
      float *dp = sld(D.p);
      const V4 p = ld4(dp + j);
      V4 pn;
#pragma unroll
      for (int e = 0; e < 4; ++e) pn.v[e] = c1 * y.v[e] - c2 * p.v[e];
      st4(dp + j, pn);
      break;
    }
    case EPI_ADJ_INIT: {
      const float su = (float)sc[SC_SU];
      V4 pn;
#pragma unroll
      for (int e = 0; e < 4; ++e) pn.v[e] = su * y.v[e];
      st4(sld(D.p) + j, pn);
      break;
    }
    case EPI_RESID: {
      const float *g = sld(D.g);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double r = (double)g[j + e] - (double)y.v[e];
        dot += r * r;
      }
      break;
    }
    default: st4(out + j, y); break;
  }
}

// The block's partial (bx: the block's index within its instance).
__device__ __forceinline__ void block_partial(const InstDesc &D, int epi, double dot, int bx) {
  if (epi == EPI_FWD || epi == EPI_RESID) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[bx] = dot;
  }
}

// The epilogue operand of output j (u for EPI_FWD, p for EPI_ADJ, g for EPI_RESID), loaded
// ahead of time so that its latency overlaps the input loads; epilogue_pre then does
// epilogue()'s arithmetic with it.
__device__ __forceinline__ const float *pre_operand(const InstDesc &D, int epi) {
  return epi == EPI_FWD ? sld(D.u) : epi == EPI_ADJ ? sld(D.p) : epi == EPI_RESID ? sld(D.g) : nullptr;
}

__device__ __forceinline__ void epilogue_pre(const InstDesc &D, int epi, long long j, float y,
                                             float pre, float *out, double &dot) {
  const double *sc = sld(D.sc);
  switch (epi) {
    case EPI_FWD: {
      const float c1 = (float)sc[SC_SV], c2 = (float)(sc[SC_ALPHA] * sc[SC_SU]);
      const float un = c1 * y - c2 * pre;
      sld(D.u)[j] = un;
      dot = (double)un * (double)un;
      break;
    }
    case EPI_ADJ: {
      const float c1 = (float)sc[SC_SU], c2 = (float)(sc[SC_BETA] * sc[SC_SV]);
      sld(D.p)[j] = c1 * y - c2 * pre;
      break;
    }
    case EPI_ADJ_INIT: sld(D.p)[j] = (float)sc[SC_SU] * y; break;
    case EPI_RESID: {
      const double e = (double)pre - (double)y;
      dot = e * e;
      break;
    }
    default: out[j] = y; break;
  }
}


}  // namespace

// x pass, any nx: a block owns kXTile consecutive voxels in linear order (rows of length nx back to
// back), 4 per thread, and stages [j0 - r, j0 + kXTile + r) in LDS; a neighbour j + k belongs
// to the same row iff 0 <= x + k < nx, which the tap range below enforces.
constexpr int kXTile = 4 * kBlock;
__global__ void __launch_bounds__(kBlock) k_blur_x(InstDesc *const *descs, int src_sel, int dst_sel,
                                                  int adj, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  __shared__ float tile[kXTile + 2 * PLSQR_MAX_RADIUS];
  __shared__ float w[kMaxTaps];
  const int r = sld(D.radius);
  const long long n = sld(D.n);
  const long long j0 = (long long)blockIdx.x * kXTile;
  double dot = 0.0;
  if (j0 < n) {
    const float *__restrict__ src = vec_of(D, src_sel);
    if (threadIdx.x < 2 * r + 1) w[threadIdx.x] = D.taps[adj ? 2 * r - threadIdx.x : threadIdx.x];
    float v[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int i = threadIdx.x + u * kBlock;
      const long long q = j0 - r + i;
      v[u] = (i < kXTile + 2 * r && q >= 0 && q < n) ? src[q] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int i = threadIdx.x + u * kBlock;
      if (i < kXTile + 2 * r) tile[i] = v[u];
    }
    __syncthreads();
    float *dst = vec_of(D, dst_sel);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + u * kBlock;
      const long long j = j0 + i;
      if (j < n) {
        const int nx = sld(D.nx);
        const int x = (int)((unsigned)j % (unsigned)nx);
        const int klo = -min(r, x), khi = min(r, nx - 1 - x);
        float y = 0.f;
        for (int k = klo; k <= khi; ++k) y += w[r + k] * tile[i + r + k];
        double dq = 0.0;
        epilogue(D, epi, j, y, dst, dq);
        dot += dq;
      }
    }
  } else {
    __syncthreads();
  }
  if (epi == EPI_FWD || epi == EPI_RESID) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
  }
}


// The radius is a template parameter of the pass bodies below: with it every window, tap loop
// and boundary test is static, so a thread's loads are straight-line code issued back to back
// (no branch per load, no wait between them) and the taps sit in scalar registers. Instances of
// one batch may differ in radius, so each block picks its body with a switch on r.
#define PLSQR_RADIUS_SWITCH(r, CALL) \
  switch (r) {                        \
    case 0: CALL(0); break;           \
    case 1: CALL(1); break;           \
    case 2: CALL(2); break;           \
    case 3: CALL(3); break;           \
    case 4: CALL(4); break;           \
    case 5: CALL(5); break;           \
    case 6: CALL(6); break;           \
    case 7: CALL(7); break;           \
    case 8: CALL(8); break;           \
    case 9: CALL(9); break;           \
    case 10: CALL(10); break;         \
    case 11: CALL(11); break;         \
    case 12: CALL(12); break;         \
    case 13: CALL(13); break;         \
    case 14: CALL(14); break;         \
    case 15: CALL(15); break;         \
    default: CALL(16); break;         \
  }
static_assert(PLSQR_MAX_RADIUS == 16, "the radius switch covers 0..16");

// zero_pad_note: inputs outside the grid are read from the nearest inside address and scaled
// by 0 rather than selected away, so that no load depends on a condition and a thread issues
// all its loads back to back. For finite data v * 0 = +-0 and v * 1 = v exactly, so the
// outputs equal those of explicit zero padding bit for bit; a non-finite boundary value that
// is copied this way only reaches outputs whose windows already contain it (the copies sit
// next to it), so NaN/Inf propagate as they would anyway.

// x pass, nx a multiple of 4: every thread computes kXG (1, 2 or 4) groups of 4 consecutive
// outputs of one
// row (fewer at the row's end) from a register window of float4 groups loaded straight from
// memory, [x0 - R4, x0 + 4 kXG + R4) with R4 = R rounded up to a multiple of 4 (groups outside
// the row are zeros: the operator's zero boundary). Out-of-row groups are loaded from a clamped
// address and replaced by zeros, so the loads carry no branches. Per output the taps are
// applied in order k = 0..2R.
template <int kXG, int R>
__device__ __forceinline__ void xg_outputs(const float *__restrict__ src, const float *T,
                                           long long rowbase, int x0, int nx, V4 (&y)[kXG]) {
  constexpr int R4 = (R + 3) & ~3;
  constexpr int kShift = R4 - R;
  constexpr int NG = kXG + R4 / 2;
  float win[4 * NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int xs = x0 - R4 + 4 * g;
    const float okf = (xs >= 0 && xs < nx) ? 1.f : 0.f;
    const int xc = min(max(xs, 0), nx - 4);
    const V4 v = ld4(src + rowbase + xc);
#pragma unroll
    for (int e = 0; e < 4; ++e) win[4 * g + e] = v.v[e] * okf;   // see zero_pad_note
  }
  float w[2 * R + 1];
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) w[k] = sld(T[k]);
#pragma unroll
  for (int g = 0; g < kXG; ++g) y[g] = V4{};
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k)
#pragma unroll
    for (int e = 0; e < 4 * kXG; ++e) y[e / 4].v[e % 4] += w[k] * win[kShift + e + k];
}

// The pending f, w update at voxel j (SC_UPD: f += (phi/rho) w, w = v / alpha - (theta/rho) w,
// the arithmetic of k_update_fw), v_j given.
__device__ __forceinline__ void update_at(float *f, float *w, long long j, float vj, float cf,
                                          float cw, float sv) {
  const float wj = w[j];
  f[j] += cf * wj;
  w[j] = sv * vj - cw * wj;
}

// Partial count of the finaliser block's instance i: fin_np.count[e] for fin_np.inst[e] == i
// (a ragged launch), else fin_n.
__device__ __forceinline__ int fin_parts(int i, int fin_n, const Rag &fin_np) {
  if (fin_np.n == 0) return fin_n;
  int c = 0;
  for (int e = 0; e < fin_np.n; ++e)
    if (fin_np.inst[e] == i) c = fin_np.count[e];
  return c;
}

// upd: also apply a pending f, w update (update_at) to this thread's output voxels; the pass
// reads v, and f and w are not touched by the product. fin >= 0: the last block of each
// instance is a finaliser block instead (fin_block with its fin_parts partials, from the
// launch before): the first pass of a product reads none of the scalars a finaliser writes.
template <int kXG>
__global__ void __launch_bounds__(kBlock) k_blur_xg(InstDesc *const *descs, int src_sel,
                                                   int dst_sel, int adj, int epi, Rag rg, int upd,
                                                   int fin, int fin_n, Rag fin_np) {
  const Blk k = locate(rg);
  if (k.i < 0) return;
  const InstDesc &D = *descs[k.i];
  if (fin >= 0 && k.bx == k.gx - 1) {
    fin_block(D, fin_parts(k.i, fin_n, fin_np), fin);
    return;
  }
  if (product_masked(D, epi)) return;
  const int r = sld(D.radius);
  const int nx = sld(D.nx);
  const long long n = sld(D.n);
  const int tpr = (nx + 4 * kXG - 1) / (4 * kXG);          // threads per row
  const long long t = (long long)k.bx * kBlock + threadIdx.x;
  const long long rows = n / nx;
  double dot = 0.0;
  if (t < rows * tpr) {
    const long long row = t / tpr;
    const int x0 = (int)(t % tpr) * 4 * kXG;
    const long long rowbase = row * nx;
    const float *__restrict__ src = vec_of(D, src_sel);
    const float *T = adj ? D.taps_rev : D.taps;
    V4 y[kXG];
#define PLSQR_XG(RR) xg_outputs<kXG, RR>(src, T, rowbase, x0, nx, y)
    PLSQR_RADIUS_SWITCH(r, PLSQR_XG)
#undef PLSQR_XG
    float *dst = vec_of(D, dst_sel);
#pragma unroll
    for (int g = 0; g < kXG; ++g)
      if (x0 + 4 * g < nx) epilogue4(D, epi, rowbase + x0 + 4 * g, y[g], dst, dot);
    const double *sc = sld(D.sc);
    if (upd && sc[SC_UPD] != 0.0 && sc[SC_STOP] == 0.0) {
      const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW], sv = (float)sc[SC_SV];
      float *f = sld(D.f), *w = sld(D.w);
#pragma unroll
      for (int g = 0; g < kXG; ++g) {
        const long long j = rowbase + x0 + 4 * g;
        if (x0 + 4 * g < nx) {
          float4 wv = *reinterpret_cast<const float4 *>(w + j);
          float4 fv = *reinterpret_cast<const float4 *>(f + j);
          const float4 vv = *reinterpret_cast<const float4 *>(src + j);
          fv.x += cf * wv.x; fv.y += cf * wv.y; fv.z += cf * wv.z; fv.w += cf * wv.w;
          wv.x = sv * vv.x - cw * wv.x; wv.y = sv * vv.y - cw * wv.y;
          wv.z = sv * vv.z - cw * wv.z; wv.w = sv * vv.w - cw * wv.w;
          *reinterpret_cast<float4 *>(f + j) = fv;
          *reinterpret_cast<float4 *>(w + j) = wv;
        }
      }   // (update_at's arithmetic, four voxels at a time)
    }
  }
  block_partial(D, epi, dot, k.bx);
}

// y or z pass with a register window (any nx): every thread owns one column element (x and the
// remaining coordinate fixed) and kWinS consecutive outputs along the axis. It issues the loads
// of all its kWinS + 2R inputs and of the epilogue operands back to back -- 64 lanes read 64
// consecutive x, so each load of a wave is one coalesced row segment -- and then forms the
// outputs from registers, taps in order k = 0..2R. No LDS and no barrier; neighbouring segments
// re-read their 2R halo lines through L2.
template <int kWinS, int R>
__device__ __forceinline__ double win_outputs(const InstDesc &D, int epi,
                                              const float *__restrict__ src, float *dst,
                                              const float *pre_src, const float *T, long long base,
                                              long long sa, int a0, int na) {
  constexpr int W = kWinS + 2 * R;
  float win[W];
#pragma unroll
  for (int m = 0; m < W; ++m) {
    const int a = a0 - R + m;
    const float okf = (a >= 0 && a < na) ? 1.f : 0.f;
    const int ac = min(max(a, 0), na - 1);
    win[m] = src[base + (long long)ac * sa] * okf;   // see zero_pad_note
  }
  float pre[kWinS];
  if (pre_src) {
#pragma unroll
    for (int q = 0; q < kWinS; ++q) pre[q] = pre_src[base + (long long)min(a0 + q, na - 1) * sa];
  } else {
#pragma unroll
    for (int q = 0; q < kWinS; ++q) pre[q] = 0.f;
  }
  float w[2 * R + 1];
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) w[k] = sld(T[k]);
  float acc[kWinS];
#pragma unroll
  for (int q = 0; q < kWinS; ++q) acc[q] = 0.f;
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k)
#pragma unroll
    for (int q = 0; q < kWinS; ++q) acc[q] += w[k] * win[q + k];
  double dot = 0.0;
#pragma unroll
  for (int q = 0; q < kWinS; ++q) {
    if (a0 + q < na) {
      double dq = 0.0;
      epilogue_pre(D, epi, base + (long long)(a0 + q) * sa, acc[q], pre[q], dst, dq);
      dot += dq;
    }
  }
  return dot;
}

// upd: also apply a pending f, w update (update_at) to this thread's output voxels (the forward
// product's second pass when the first carries a finaliser block).
template <int kWinS>
__global__ void __launch_bounds__(kBlock) k_blur_win(InstDesc *const *descs, int axis,
                                                    int src_sel, int dst_sel, int adj, int epi,
                                                    Rag rg, int upd) {
  const Blk k = locate(rg);
  if (k.i < 0) return;
  const InstDesc &D = *descs[k.i];
  if (product_masked(D, epi)) return;
  const int r = sld(D.radius);
  const int nx = sld(D.nx), ny = sld(D.ny), nz = sld(D.nz);
  const int na = (axis == 1) ? ny : nz;        // extent along the pass
  const int no = (axis == 1) ? nz : ny;        // the remaining coordinate
  const long long sa = (axis == 1) ? (long long)nx : (long long)nx * ny;
  const long long so = (axis == 1) ? (long long)nx * ny : (long long)nx;
  const int segs = (na + kWinS - 1) / kWinS;
  const long long total = (long long)nx * segs * no;
  // consecutive segments of a line share 2R halo lines: xcd_tile keeps consecutive blocks on
  // one XCD, so the halo is re-read from that XCD's L2
  const long long t = xcd_tile_of(k) * kBlock + threadIdx.x;
  double dot = 0.0;
  if (t < total) {
    const int x = (int)(t % nx);
    const long long rest = t / nx;
    const int seg = (int)(rest % segs);
    const int o = (int)(rest / segs);
    const long long base = (long long)o * so + x;
    const float *T = adj ? D.taps_rev : D.taps;
    const float *__restrict__ src = vec_of(D, src_sel);
    float *dst = vec_of(D, dst_sel);
    const float *pre_src = pre_operand(D, epi);
#define PLSQR_WIN(RR) dot = win_outputs<kWinS, RR>(D, epi, src, dst, pre_src, T, base, sa, seg * kWinS, na)
    PLSQR_RADIUS_SWITCH(r, PLSQR_WIN)
#undef PLSQR_WIN
    const double *sc = sld(D.sc);
    if (upd && sc[SC_UPD] != 0.0 && sc[SC_STOP] == 0.0) {
      const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW], sv = (float)sc[SC_SV];
      float *f = sld(D.f), *w = sld(D.w);
      const float *v = sld(D.v);
      const int a0 = seg * kWinS;
      float vq[kWinS];
#pragma unroll
      for (int q = 0; q < kWinS; ++q) vq[q] = (a0 + q < na) ? v[base + (long long)(a0 + q) * sa] : 0.f;
#pragma unroll
      for (int q = 0; q < kWinS; ++q)
        if (a0 + q < na) update_at(f, w, base + (long long)(a0 + q) * sa, vq[q], cf, cw, sv);
    }
  }
  block_partial(D, epi, dot, k.bx);
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
#define LAUNCH_B(kern, gx, gy, ...) \
  hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kBlock), 0, st, __VA_ARGS__)

// Work per thread of the blur passes when not set by the caller: measured on 128^3 grids, alone
// and in lockstep batches of 8, 2 groups per thread in x and 8 outputs per thread along y and z
// are within a few percent of the best of {1, 2, 4} x {4, 8, 16, 32}.
constexpr int kDefaultXGroups = 2;
constexpr int kDefaultWindow = 8;

int blur_x_blocks(long long n, int nx, int groups) {
  if (nx % 4 != 0) return (int)((n + kXTile - 1) / kXTile);
  const int G = groups ? groups : kDefaultXGroups;
  const long long threads = n / nx * ((nx + 4 * G - 1) / (4 * G));
  return (int)((threads + kBlock - 1) / kBlock);
}
int blur_axis_blocks(int nx, int ny, int nz, int axis, int window) {
  const int S = window ? window : kDefaultWindow;
  const int na = (axis == 1) ? ny : nz, no = (axis == 1) ? nz : ny;
  const long long threads = (long long)nx * ((na + S - 1) / S) * no;
  return (int)((threads + kBlock - 1) / kBlock);
}

// Grid of a launch: (g, B) for a uniform launch, (the ragged map's extent, 1) for a ragged one.
static dim3 grid_of(unsigned g, int B, const Rag &rg) {
  if (rg.n == 0) return dim3(g, B);
  return dim3((unsigned)(rg.first[rg.n - 1] + rg.count[rg.n - 1]), 1);
}

int launch_blur_x(hipStream_t st, InstDesc *const *d, int B, long long n, int nx, int src, int dst,
                  int adj, int epi, int groups, const Rag &rg, int upd, int fin, int fin_n,
                  const Rag &fin_np) {
  const unsigned g = (unsigned)blur_x_blocks(n, nx, groups);
  // a uniform launch's finaliser blocks: one more block per instance (a ragged map counts them)
  const dim3 grid = grid_of(fin >= 0 ? g + 1 : g, B, rg);
  if (nx % 4 == 0) {
    const int G = groups ? groups : kDefaultXGroups;
    if (G == 1)
      hipLaunchKernelGGL(k_blur_xg<1>, grid, dim3(kBlock), 0, st, d, src, dst, adj, epi, rg, upd,
                         fin, fin_n, fin_np);
    else if (G == 2)
      hipLaunchKernelGGL(k_blur_xg<2>, grid, dim3(kBlock), 0, st, d, src, dst, adj, epi, rg, upd,
                         fin, fin_n, fin_np);
    else
      hipLaunchKernelGGL(k_blur_xg<4>, grid, dim3(kBlock), 0, st, d, src, dst, adj, epi, rg, upd,
                         fin, fin_n, fin_np);
    return (int)g;
  }
  LAUNCH_B(k_blur_x, g, B, d, src, dst, adj, epi);   // uniform launches only (see the driver)
  return (int)g;
}
int launch_blur_axis(hipStream_t st, InstDesc *const *d, int B, int nx, int ny, int nz, int axis,
                     int src, int dst, int adj, int epi, int window, const Rag &rg, int upd) {
  const int S = window ? window : kDefaultWindow;
  const unsigned g = (unsigned)blur_axis_blocks(nx, ny, nz, axis, window);
  const dim3 grid = grid_of(g, B, rg);
  if (S == 4)
    hipLaunchKernelGGL(k_blur_win<4>, grid, dim3(kBlock), 0, st, d, axis, src, dst, adj, epi, rg, upd);
  else if (S == 8)
    hipLaunchKernelGGL(k_blur_win<8>, grid, dim3(kBlock), 0, st, d, axis, src, dst, adj, epi, rg, upd);
  else if (S == 32)
    hipLaunchKernelGGL(k_blur_win<32>, grid, dim3(kBlock), 0, st, d, axis, src, dst, adj, epi, rg, upd);
  else
    hipLaunchKernelGGL(k_blur_win<16>, grid, dim3(kBlock), 0, st, d, axis, src, dst, adj, epi, rg, upd);
  return (int)g;
}

}  // namespace plsqr
