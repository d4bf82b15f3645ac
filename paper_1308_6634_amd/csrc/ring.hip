// Matrix-free source-detector sensitivity: the dense operator of the ring workloads applied
// without storing it. Entry (s * n_det + d, j) is
//     exp(-mu (r_sj + r_dj)) / (r_sj r_dj + 1) = a_s(j) c_d(j) / (r_sj r_dj + 1),
// with r_sj, r_dj the distances from voxel centre j to source s and detector d and
// a_s = exp(-mu r_sj), c_d = exp(-mu r_dj). The method needs only the action of A and A^T
// (Section 1: the forward map is available by its action; in Section 5 each application is a
// set of PDE solves). Each product regenerates every entry, so it is bound by ALU work, not by
// HBM: per entry one FMA (r_s r_d + 1), one reciprocal, one multiply and one FMA; the
// exponentials and square roots are per (point, voxel) pair and are shared by a whole row or
// column of entries.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

namespace {

constexpr int kRingTile = 64;   // sources and detectors per forward tile (4 x 4 per thread)
constexpr int kRingSub = 32;    // voxels staged per step of the forward product
constexpr int kRingDet = 16;    // detectors held in registers per pass of the adjoint

__device__ __forceinline__ void voxel_xyz(long long j, int nx, int ny, float &x, float &y,
                                          float &z) {
  const unsigned jj = (unsigned)j, q = jj / (unsigned)nx;   // grids hold < 2^31 cells
  x = (float)(jj - q * (unsigned)nx);
  y = (float)(q % (unsigned)ny);
  z = (float)(q / (unsigned)ny);
}

__device__ __forceinline__ float point_dist(const float *p, float x, float y, float z) {
  const float dx = x - p[0], dy = y - p[1], dz = z - p[2];
  return __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
}

// The same for a point every lane reads (the positions are written once by the host, so they
// may be read through the scalar cache).
__device__ __forceinline__ float point_dist_u(const float *p, float x, float y, float z) {
  const float dx = x - sld(p[0]), dy = y - sld(p[1]), dz = z - sld(p[2]);
  return __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
}

// 1/t for t >= 1 (the hardware reciprocal, ~1 ulp)
__device__ __forceinline__ float rcp(float t) { return __builtin_amdgcn_rcpf(t); }

}  // namespace

// Forward product, split over voxel chunks: block (tile, chunk) accumulates, for its 64 x 64
// tile of (source, detector) rows, sum_j A(sd, j) v_j over the chunk's voxels into
// ringpart[chunk][row]. Per 32-voxel step the block stages a_s, r_s for its 64 sources and
// c_d, r_d for its 64 detectors (16 (distance, exponential) pairs per thread) and v in LDS;
// every thread then forms its 4 x 4 entries for each voxel in voxel order.
__global__ void __launch_bounds__(kBlock) k_ring_fwd(InstDesc *const *descs, int src_sel, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  __shared__ __align__(16) float sa[kRingSub][kRingTile], sr[kRingSub][kRingTile];
  __shared__ __align__(16) float dc[kRingSub][kRingTile], dr[kRingSub][kRingTile];
  __shared__ float vs[kRingSub], vx[kRingSub], vy[kRingSub], vz[kRingSub];
  const int ns = sld(D.n_src), nd = sld(D.n_det);
  const int nx = sld(D.nx), ny = sld(D.ny);
  const long long n = sld(D.n);
  const int chunk = sld(D.ring_chunk);
  const float mu = sld(D.ring_mu);
  const float *geo = sld(D.ring);
  const int dt_n = (nd + kRingTile - 1) / kRingTile;
  const int tiles = ((ns + kRingTile - 1) / kRingTile) * dt_n;
  const int tile = (int)(blockIdx.x % tiles);
  const long long c = blockIdx.x / tiles;
  const int s0 = (tile / dt_n) * kRingTile, d0 = (tile % dt_n) * kRingTile;
  const long long j0 = c * chunk, j1 = min(n, j0 + chunk);
  const float *__restrict__ v = vec_of(D, src_sel);
  const int ts = threadIdx.x / 16, td = threadIdx.x % 16;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[i][k] = 0.f;
  for (long long jb = j0; jb < j1; jb += kRingSub) {
    if (threadIdx.x < kRingSub) {
      const long long j = jb + threadIdx.x;
      float x = 0.f, y = 0.f, z = 0.f;
      if (j < j1) voxel_xyz(j, nx, ny, x, y, z);
      vx[threadIdx.x] = x;
      vy[threadIdx.x] = y;
      vz[threadIdx.x] = z;
      vs[threadIdx.x] = j < j1 ? v[j] : 0.f;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * kRingTile * kRingSub; q += kBlock) {
      const int p = q % kRingTile, jj = (q / kRingTile) % kRingSub;
      const bool det = q >= kRingTile * kRingSub;
      const long long j = jb + jj;
      const int idx = (det ? d0 : s0) + p;
      float e = 0.f, r = 0.f;
      if (idx < (det ? nd : ns) && j < j1) {
        r = point_dist(geo + (det ? 3 * ns : 0) + 3 * idx, vx[jj], vy[jj], vz[jj]);
        e = __expf(-mu * r);
      }
      if (det) {
        dc[jj][p] = e;
        dr[jj][p] = r;
      } else {
        sa[jj][p] = e;
        sr[jj][p] = r;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < kRingSub; ++jj) {
      const float vj = vs[jj];
      const float4 a4 = *reinterpret_cast<const float4 *>(&sa[jj][4 * ts]);
      const float4 r4 = *reinterpret_cast<const float4 *>(&sr[jj][4 * ts]);
      const float4 c4 = *reinterpret_cast<const float4 *>(&dc[jj][4 * td]);
      const float4 e4 = *reinterpret_cast<const float4 *>(&dr[jj][4 * td]);
      const float av[4] = {a4.x * vj, a4.y * vj, a4.z * vj, a4.w * vj};
      const float rs[4] = {r4.x, r4.y, r4.z, r4.w};
      const float cd[4] = {c4.x, c4.y, c4.z, c4.w};
      const float rd[4] = {e4.x, e4.y, e4.z, e4.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          acc[i][k] = fmaf(av[i] * cd[k], rcp(fmaf(rs[i], rd[k], 1.f)), acc[i][k]);
    }
    __syncthreads();
  }
  float *part = sld(D.ringpart) + c * sld(D.m);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int s = s0 + 4 * ts + i;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = d0 + 4 * td + k;
      if (s < ns && d < nd) part[(long long)s * nd + d] = acc[i][k];
    }
  }
}

// First stage of the sum over chunks: block (row block, group g) sums, for each of its rows,
// the partials of chunks [g * per, (g + 1) * per) in chunk order into ringpart2[g][row]
// (loads issued 8 at a time, additions in order).
__global__ void __launch_bounds__(kBlock) k_ring_fwd_sum(InstDesc *const *descs, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  const long long m = sld(D.m);
  const int rblocks = (int)((m + kBlock - 1) / kBlock);
  const int g = blockIdx.x / rblocks;
  const long long row = (long long)(blockIdx.x % rblocks) * kBlock + threadIdx.x;
  if (row >= m) return;
  const int chunks = sld(D.ring_chunks), groups = sld(D.ring_groups);
  const int per = (chunks + groups - 1) / groups;
  const int c0 = g * per, c1 = min(chunks, c0 + per);
  const float *part = sld(D.ringpart);
  float y = 0.f;
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    float t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = part[(long long)(c + i) * m + row];
#pragma unroll
    for (int i = 0; i < 8; ++i) y += t[i];
  }
  for (; c < c1; ++c) y += part[(long long)c * m + row];
  sld(D.ringpart2)[(long long)g * m + row] = y;
}

// Second stage: the group sums of each row in group order, then the product's epilogue.
__global__ void __launch_bounds__(kBlock) k_ring_fwd_reduce(InstDesc *const *descs, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  const long long m = sld(D.m);
  const long long row = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (row < m) {
    const float *p2 = sld(D.ringpart2);
    const int groups = sld(D.ring_groups);
    float y = 0.f;
    for (int g = 0; g < groups; ++g) y += p2[(long long)g * m + row];
    epilogue(D, epi, row, y, nullptr, dot);
  }
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

// Adjoint product: one thread per voxel j, A^T u at j = sum_s a_s(j) sum_d c_d(j) u_sd /
// (r_sj r_dj + 1). u (n_Y <= 16384 floats) is staged in LDS and read by all lanes at the same
// address; detectors go through registers 16 at a time, sources are visited in order for each
// group.
__global__ void __launch_bounds__(kBlock) k_ring_adj(InstDesc *const *descs, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  extern __shared__ __align__(16) float su[];
  const long long m = sld(D.m);
  const float *__restrict__ u = sld(D.u);
  for (long long i = threadIdx.x; i < m; i += kBlock) su[i] = u[i];
  __syncthreads();
  const int ns = sld(D.n_src), nd = sld(D.n_det);
  const int nx = sld(D.nx), ny = sld(D.ny);
  const long long n = sld(D.n);
  const float mu = sld(D.ring_mu);
  const float *geo = sld(D.ring);
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  float x, y, z;
  voxel_xyz(j, nx, ny, x, y, z);
  float acc = 0.f;
  for (int g0 = 0; g0 < nd; g0 += kRingDet) {
    float cd[kRingDet], rd[kRingDet];
#pragma unroll
    for (int k = 0; k < kRingDet; ++k) {
      cd[k] = 0.f;
      rd[k] = 0.f;
      if (g0 + k < nd) {
        rd[k] = point_dist_u(geo + 3 * ns + 3 * (g0 + k), x, y, z);
        cd[k] = __expf(-mu * rd[k]);
      }
    }
    const int kn = min(kRingDet, nd - g0);
    // whole groups of 16 on 16-byte aligned rows: u read as float4
    const bool vec = kn == kRingDet && (nd & 3) == 0;
    for (int s = 0; s < ns; ++s) {
      const float rs = point_dist_u(geo + 3 * s, x, y, z);
      const float as = __expf(-mu * rs);
      const float *us = su + (long long)s * nd + g0;
      float uk[kRingDet];
      if (vec) {
#pragma unroll
        for (int q = 0; q < kRingDet / 4; ++q) {
          const float4 t4 = reinterpret_cast<const float4 *>(us)[q];
          uk[4 * q] = t4.x;
          uk[4 * q + 1] = t4.y;
          uk[4 * q + 2] = t4.z;
          uk[4 * q + 3] = t4.w;
        }
      } else {
#pragma unroll
        for (int k = 0; k < kRingDet; ++k) uk[k] = k < kn ? us[k] : 0.f;
      }
      float t = 0.f;
#pragma unroll
      for (int k = 0; k < kRingDet; ++k) t = fmaf(cd[k] * uk[k], rcp(fmaf(rs, rd[k], 1.f)), t);
      acc = fmaf(as, t, acc);
    }
  }
  double unused = 0.0;
  epilogue(D, epi, j, acc, nullptr, unused);
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
int launch_ring_forward(hipStream_t st, InstDesc *const *d, int B, const InstDesc &H, int src,
                        int epi) {
  const int tiles = ((H.n_src + kRingTile - 1) / kRingTile) * ((H.n_det + kRingTile - 1) / kRingTile);
  hipLaunchKernelGGL(k_ring_fwd, dim3((unsigned)(tiles * H.ring_chunks), B), dim3(kBlock), 0, st,
                     d, src, epi);
  const unsigned rb = (unsigned)((H.m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_ring_fwd_sum, dim3(rb * (unsigned)H.ring_groups, B), dim3(kBlock), 0, st, d,
                     epi);
  hipLaunchKernelGGL(k_ring_fwd_reduce, dim3(rb, B), dim3(kBlock), 0, st, d, epi);
  return (int)rb;
}

void launch_ring_adjoint(hipStream_t st, InstDesc *const *d, int B, const InstDesc &H, int epi) {
  const unsigned g = (unsigned)((H.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_ring_adj, dim3(g, B), dim3(kBlock), (size_t)H.m * sizeof(float), st, d,
                     epi);
}

}  // namespace plsqr
