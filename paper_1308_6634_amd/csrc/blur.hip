// Separable Gaussian blur, the structured forward operator A of the test problems (and its
// adjoint, the same passes with reversed taps): one 1D correlation pass per axis with zero
// values outside the grid, y[x] = sum_k w[k] src[x + k - r]. The last pass applies the Krylov
// epilogue of the bidiagonalization (section 3.2, Algorithm 2). Every pass reads and writes
// one vector, so the passes are HBM-bound; the kernels below keep each HBM byte read once
// (halo re-reads come from L1/LDS) and move data in 16-byte vectors where the rows allow.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
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

__device__ __forceinline__ void block_partial(const InstDesc &D, int epi, double dot) {
  if (epi == EPI_FWD || epi == EPI_RESID) {
    dot = block_sum(dot);
    if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
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

// Tile handled by this block. Workgroups are dealt to the 8 XCDs round-robin; when the grid
// splits evenly, consecutive tiles are given to blocks on the same XCD, so the halo rows that
// neighbouring tiles share are found in that XCD's L2.
__device__ __forceinline__ long long xcd_tile() {
  const unsigned b = blockIdx.x, nb = gridDim.x;
  if (nb % 8u != 0u) return b;
  return (long long)(b % 8u) * (nb / 8u) + b / 8u;
}

constexpr int kR4Max = (PLSQR_MAX_RADIUS + 3) / 4 * 4;   // radius rounded up to a multiple of 4
constexpr int kWinGroups = 1 + kR4Max / 2;               // float4 groups in a 4-output window
constexpr int kWin = 4 * kWinGroups + 4;                 // + 4 zeros: every unrolled index valid

}  // namespace

// x pass, any nx: a block owns kXTile consecutive voxels in linear order (rows of length nx back to
// back), 4 per thread, and stages [j0 - r, j0 + kXTile + r) in LDS; a neighbour j + k belongs
// to the same row iff 0 <= x + k < nx, which the tap range below enforces.
constexpr int kXTile = 4 * kBlock;
__global__ void __launch_bounds__(kBlock) k_blur_x(InstDesc *const *descs, int src_sel, int dst_sel,
                                                  int adj, int epi) {
  const InstDesc &D = inst(descs);
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


// x pass, nx a multiple of 4: every thread computes the 4 outputs x0..x0+3 (x0 % 4 == 0) of one
// row from a register window [x0 - R4, x0 + 4 + R4), R4 = r rounded up to a multiple of 4,
// loaded as float4 groups straight from memory (neighbouring threads' windows overlap in L1).
// A group lies wholly inside or wholly outside the row; outside groups are zeros, which is the
// operator's zero boundary. kShift = R4 - r places tap k of output e at window index
// kShift + e + k.
template <int kShift>
__device__ __forceinline__ V4 blur_x_window(const float *__restrict__ src, const float *w,
                                            long long j, int x0, int nx, int r) {
  const int R4 = r + kShift;
  const int ng = 1 + R4 / 2;
  const int ntaps = 2 * r + 1;
  float win[kWin];
#pragma unroll
  for (int g = 0; g < kWinGroups; ++g) {
    const int xs = x0 - R4 + 4 * g;
    V4 v = {};
    if (g < ng && xs >= 0 && xs < nx) v = ld4(src + j - R4 + 4 * g);
#pragma unroll
    for (int e = 0; e < 4; ++e) win[4 * g + e] = v.v[e];
  }
#pragma unroll
  for (int e = 4 * kWinGroups; e < kWin; ++e) win[e] = 0.f;
  V4 y = {};
#pragma unroll
  for (int k = 0; k < kMaxTaps; ++k) {
    if (k < ntaps) {
      const float wk = w[k];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (kShift + e + k < kWin) y.v[e] += wk * win[kShift + e + k];
    }
  }
  return y;
}

// The radius is per instance (instances of one batch may differ), so the window offset is
// selected per block.
__global__ void __launch_bounds__(kBlock) k_blur_x4(InstDesc *const *descs, int src_sel,
                                                   int dst_sel, int adj, int epi) {
  const InstDesc &D = inst(descs);
  __shared__ float w[kMaxTaps];
  const int r = sld(D.radius);
  if (threadIdx.x < 2 * r + 1) w[threadIdx.x] = D.taps[adj ? 2 * r - threadIdx.x : threadIdx.x];
  __syncthreads();
  const long long j = 4 * ((long long)blockIdx.x * kBlock + threadIdx.x);
  double dot = 0.0;
  if (j < sld(D.n)) {
    const int nx = sld(D.nx);
    const int x0 = (int)((unsigned)j % (unsigned)nx);
    const float *__restrict__ src = vec_of(D, src_sel);
    V4 y;
    switch ((4 - r % 4) % 4) {
      case 0: y = blur_x_window<0>(src, w, j, x0, nx, r); break;
      case 1: y = blur_x_window<1>(src, w, j, x0, nx, r); break;
      case 2: y = blur_x_window<2>(src, w, j, x0, nx, r); break;
      default: y = blur_x_window<3>(src, w, j, x0, nx, r); break;
    }
    epilogue4(D, epi, j, y, vec_of(D, dst_sel), dot);
  }
  block_partial(D, epi, dot);
}

// y or z pass: a block of 64 x 4 threads owns a strip of 64 x-columns and kStripA outputs along
// the axis (the other coordinate fixed). It stages the kStripA + 2r input planes of the strip in
// LDS (16-byte loads when nx is a multiple of 4), then each thread computes kStripA / 4
// consecutive outputs of one column from a window of LDS values read once each; the tap
// products are accumulated per output in tap order, out-of-grid planes being zeros.
constexpr int kStripX = 64;
template <int kStripA>
__global__ void __launch_bounds__(kBlock) k_blur_strip(InstDesc *const *descs, int axis,
                                                      int src_sel, int dst_sel, int adj, int epi) {
  constexpr int kOut = kStripA / 4;
  const InstDesc &D = inst(descs);
  __shared__ float tile[kStripA + 2 * PLSQR_MAX_RADIUS][kStripX];
  __shared__ float w[kMaxTaps];
  const int r = sld(D.radius);
  const int nx = sld(D.nx), ny = sld(D.ny), nz = sld(D.nz);
  const int na = (axis == 1) ? ny : nz;        // extent along the pass
  const int no = (axis == 1) ? nz : ny;        // the remaining coordinate
  const long long sa = (axis == 1) ? (long long)nx : (long long)nx * ny;
  const long long so = (axis == 1) ? (long long)nx * ny : (long long)nx;
  const int tx_n = (nx + kStripX - 1) / kStripX, ta_n = (na + kStripA - 1) / kStripA;
  const long long tiles = (long long)tx_n * ta_n * no;
  const long long t = xcd_tile();
  const int lx = threadIdx.x & (kStripX - 1), la = threadIdx.x / kStripX;   // 64 x 4
  if (threadIdx.x < 2 * r + 1) w[threadIdx.x] = D.taps[adj ? 2 * r - threadIdx.x : threadIdx.x];
  int tx = 0, ta = 0, o = 0;
  if (t < tiles) {
    tx = (int)(t % tx_n);
    const long long rest = t / tx_n;
    ta = (int)(rest % ta_n);
    o = (int)(rest / ta_n);
  }
  const int a0 = ta * kStripA;
  const int rows = kStripA + 2 * r;
  const float *__restrict__ src = vec_of(D, src_sel);
  const long long obase = (long long)o * so;
  if (t < tiles) {
    if ((nx & 3) == 0) {
      // 16 float4 columns x 16 planes per pass of the block, 4 loads in flight per thread
      const int c4 = threadIdx.x & 15, sub = threadIdx.x >> 4;
      const int xg = tx * kStripX + 4 * c4;
      for (int i0 = sub; i0 < rows; i0 += 64) {
        V4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 16 * u;
          const int a = a0 - r + i;
          v[u] = V4{};
          if (i < rows && xg < nx && a >= 0 && a < na) v[u] = ld4(src + obase + xg + (long long)a * sa);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 16 * u;
          if (i < rows)
            *reinterpret_cast<float4 *>(&tile[i][4 * c4]) =
                make_float4(v[u].v[0], v[u].v[1], v[u].v[2], v[u].v[3]);
        }
      }
    } else {
      const int x = tx * kStripX + lx;
      for (int i0 = la; i0 < rows; i0 += 16) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 4 * u;
          const int a = a0 - r + i;
          v[u] = (i < rows && x < nx && a >= 0 && a < na) ? src[obase + x + (long long)a * sa] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 4 * u;
          if (i < rows) tile[i][lx] = v[u];
        }
      }
    }
  }
  const int x = tx * kStripX + lx;
  const long long base = obase + x;
  const float *pre_src = pre_operand(D, epi);
  float pre[kOut];
#pragma unroll
  for (int q = 0; q < kOut; ++q) {
    const int a = a0 + la * kOut + q;
    pre[q] = (pre_src && t < tiles && x < nx && a < na) ? pre_src[base + (long long)a * sa] : 0.f;
  }
  __syncthreads();
  double dot = 0.0;
  if (t < tiles && x < nx) {
    const int q0 = la * kOut;
    const int nwin = kOut + 2 * r;
    float acc[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) acc[q] = 0.f;
#pragma unroll
    for (int m = 0; m < kOut + 2 * PLSQR_MAX_RADIUS; ++m) {
      if (m < nwin) {
        const float v = tile[q0 + m][lx];
#pragma unroll
        for (int q = 0; q < kOut; ++q) {
          const int k = m - q;
          if (k >= 0 && k <= 2 * r) acc[q] += w[k] * v;
        }
      }
    }
    float *dst = vec_of(D, dst_sel);
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      const int a = a0 + q0 + q;
      if (a < na) {
        double dq = 0.0;
        epilogue_pre(D, epi, base + (long long)a * sa, acc[q], pre[q], dst, dq);
        dot += dq;
      }
    }
  }
  block_partial(D, epi, dot);
}

// Fused x and y passes (nx a multiple of 4, ny > 1): a block of 256 threads owns an output
// tile of kStripX x-columns by kTileY rows of one z-plane. It stages the input rows
// [y0 - r, y0 + kTileY + r) and columns [x0 - R4, x0 + kStripX + R4) in LDS (zeros outside the
// grid), runs the x pass over all those rows into a second LDS tile (4 outputs per task from a
// register window, as k_blur_x4), then the y pass from that tile (as k_blur_strip). The
// intermediate is rounded to FP32 exactly as the separate passes store it, so the result is
// the same as the x pass followed by the y pass; the intermediate never goes to HBM.
constexpr int kTileY = 16;
constexpr int kTileCols = kStripX + 2 * kR4Max;                 // staged columns
constexpr int kTileRows = kTileY + 2 * PLSQR_MAX_RADIUS;        // staged rows

template <int kShift>
__device__ __forceinline__ void xy_xphase(const float (*tile)[kTileCols], float (*mid)[kStripX],
                                          const float *w, int r, int rows) {
  const int R4 = r + kShift;
  const int ng = 1 + R4 / 2;
  const int ntaps = 2 * r + 1;
  for (int q = threadIdx.x; q < rows * (kStripX / 4); q += kBlock) {
    const int row = q / (kStripX / 4), g = q % (kStripX / 4);
    float win[kWin];
#pragma unroll
    for (int k = 0; k < kWinGroups; ++k) {
      V4 v = {};
      if (k < ng) {
        const float4 t = *reinterpret_cast<const float4 *>(&tile[row][4 * g + 4 * k]);
        v.v[0] = t.x; v.v[1] = t.y; v.v[2] = t.z; v.v[3] = t.w;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) win[4 * k + e] = v.v[e];
    }
#pragma unroll
    for (int e = 4 * kWinGroups; e < kWin; ++e) win[e] = 0.f;
    V4 y = {};
#pragma unroll
    for (int k = 0; k < kMaxTaps; ++k) {
      if (k < ntaps) {
        const float wk = w[k];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kShift + e + k < kWin) y.v[e] += wk * win[kShift + e + k];
      }
    }
    *reinterpret_cast<float4 *>(&mid[row][4 * g]) = make_float4(y.v[0], y.v[1], y.v[2], y.v[3]);
  }
}

__global__ void __launch_bounds__(kBlock) k_blur_xy(InstDesc *const *descs, int src_sel,
                                                   int dst_sel, int adj, int epi) {
  constexpr int kOut = kTileY / 4;
  const InstDesc &D = inst(descs);
  __shared__ __align__(16) float tile[kTileRows][kTileCols];
  __shared__ __align__(16) float mid[kTileRows][kStripX];
  __shared__ float w[kMaxTaps];
  const int r = sld(D.radius);
  const int nx = sld(D.nx), ny = sld(D.ny), nz = sld(D.nz);
  const int tx_n = (nx + kStripX - 1) / kStripX, ty_n = (ny + kTileY - 1) / kTileY;
  const long long tiles = (long long)tx_n * ty_n * nz;
  const long long t = xcd_tile();
  if (threadIdx.x < 2 * r + 1) w[threadIdx.x] = D.taps[adj ? 2 * r - threadIdx.x : threadIdx.x];
  int tx = 0, ty = 0, z = 0;
  if (t < tiles) {
    tx = (int)(t % tx_n);
    const long long rest = t / tx_n;
    ty = (int)(rest % ty_n);
    z = (int)(rest / ty_n);
  }
  const int x0 = tx * kStripX, y0 = ty * kTileY;
  const int R4 = (r + 3) & ~3;
  const int rows = kTileY + 2 * r;
  const int cols4 = (kStripX + 2 * R4) / 4;
  const float *__restrict__ src = vec_of(D, src_sel);
  const long long zbase = (long long)z * nx * ny;
  if (t < tiles) {
    for (int q0 = threadIdx.x; q0 < rows * cols4; q0 += 4 * kBlock) {
      V4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * kBlock;
        const int row = q / cols4, c4 = q % cols4;
        const int y = y0 - r + row, xg = x0 - R4 + 4 * c4;
        v[u] = V4{};
        if (q < rows * cols4 && y >= 0 && y < ny && xg >= 0 && xg < nx)
          v[u] = ld4(src + zbase + (long long)y * nx + xg);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * kBlock;
        if (q < rows * cols4) {
          const int row = q / cols4, c4 = q % cols4;
          *reinterpret_cast<float4 *>(&tile[row][4 * c4]) =
              make_float4(v[u].v[0], v[u].v[1], v[u].v[2], v[u].v[3]);
        }
      }
    }
  }
  const int lx = threadIdx.x & (kStripX - 1), la = threadIdx.x / kStripX;
  const int x = x0 + lx;
  const float *pre_src = pre_operand(D, epi);
  float pre[kOut];
#pragma unroll
  for (int q = 0; q < kOut; ++q) {
    const int y = y0 + la * kOut + q;
    pre[q] = (pre_src && t < tiles && x < nx && y < ny) ? pre_src[zbase + (long long)y * nx + x] : 0.f;
  }
  __syncthreads();
  if (t < tiles) {
    switch (R4 - r) {
      case 0: xy_xphase<0>(tile, mid, w, r, rows); break;
      case 1: xy_xphase<1>(tile, mid, w, r, rows); break;
      case 2: xy_xphase<2>(tile, mid, w, r, rows); break;
      default: xy_xphase<3>(tile, mid, w, r, rows); break;
    }
  }
  __syncthreads();
  double dot = 0.0;
  if (t < tiles && x < nx) {
    const int q0 = la * kOut;
    const int nwin = kOut + 2 * r;
    float acc[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) acc[q] = 0.f;
#pragma unroll
    for (int m = 0; m < kOut + 2 * PLSQR_MAX_RADIUS; ++m) {
      if (m < nwin) {
        // the x pass leaves zeros in rows outside the grid (their inputs were zeros)
        const float v = mid[q0 + m][lx];
#pragma unroll
        for (int q = 0; q < kOut; ++q) {
          const int k = m - q;
          if (k >= 0 && k <= 2 * r) acc[q] += w[k] * v;
        }
      }
    }
    float *dst = vec_of(D, dst_sel);
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      const int y = y0 + q0 + q;
      if (y < ny) {
        double dq = 0.0;
        epilogue_pre(D, epi, zbase + (long long)y * nx + x, acc[q], pre[q], dst, dq);
        dot += dq;
      }
    }
  }
  block_partial(D, epi, dot);
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
#define LAUNCH_B(kern, gx, gy, ...) \
  hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kBlock), 0, st, __VA_ARGS__)

int launch_blur_x(hipStream_t st, InstDesc *const *d, int B, long long n, int nx, int src, int dst,
                  int adj, int epi) {
  if (nx % 4 == 0) {
    const unsigned g = (unsigned)((n / 4 + kBlock - 1) / kBlock);
    LAUNCH_B(k_blur_x4, g, B, d, src, dst, adj, epi);
    return (int)g;
  }
  const unsigned g = (unsigned)((n + kXTile - 1) / kXTile);
  LAUNCH_B(k_blur_x, g, B, d, src, dst, adj, epi);
  return (int)g;
}
int launch_blur_xy(hipStream_t st, InstDesc *const *d, int B, int nx, int ny, int nz, int src,
                   int dst, int adj, int epi) {
  const long long tiles = (long long)((nx + kStripX - 1) / kStripX) * ((ny + kTileY - 1) / kTileY) * nz;
  LAUNCH_B(k_blur_xy, (unsigned)tiles, B, d, src, dst, adj, epi);
  return (int)tiles;
}
int launch_blur_strip(hipStream_t st, InstDesc *const *d, int B, int nx, int ny, int nz, int axis,
                      int src, int dst, int adj, int epi, int depth) {
  const int na = (axis == 1) ? ny : nz, no = (axis == 1) ? nz : ny;
  const long long tiles = (long long)((nx + kStripX - 1) / kStripX) * ((na + depth - 1) / depth) * no;
  if (depth == 16)
    LAUNCH_B(k_blur_strip<16>, (unsigned)tiles, B, d, axis, src, dst, adj, epi);
  else if (depth == 64)
    LAUNCH_B(k_blur_strip<64>, (unsigned)tiles, B, d, axis, src, dst, adj, epi);
  else
    LAUNCH_B(k_blur_strip<32>, (unsigned)tiles, B, d, axis, src, dst, adj, epi);
  return (int)tiles;
}

}  // namespace plsqr
