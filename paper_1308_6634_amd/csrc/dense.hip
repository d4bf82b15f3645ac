// Dense products of the forward operator A (n_Y x n_X, row-major FP32 in HBM) in FP32:
// y = A x one block per kRows rows (each row streamed once with 16-byte loads), and
// x = A^T u as column partial sums over row chunks followed by a chunk sum. Both apply the
// Krylov epilogues of the bidiagonalization (section 3.2, Algorithm 2) to their outputs.
// These are the HBM-bound kernels of the dense-operator path; a batch of instances that
// shares A uses the MFMA kernels in gemm_bf16.hip instead.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace plsqr {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Dense forward product y = A x for kRows rows per block, epilogue per row.
template <int kRows>
__global__ void __launch_bounds__(kBlock) k_gemv_rows(InstDesc *const *descs, int src_sel, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  const long long row0 = (long long)blockIdx.x * kRows;
  const long long n = sld(D.n);
  const float *__restrict__ x = vec_of(D, src_sel);
  const float *__restrict__ A = sld(D.A);
  float acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0.f;
  const int nrows = (int)min((long long)kRows, max(0LL, sld(D.m) - row0));
  if ((n & 3) == 0) {
    // Each thread walks its columns c = tid, tid + kBlock, ... in order; kUnroll column
    // groups are loaded (x once, every row of A) before any is used, so that many 16-byte
    // loads are in flight per thread. A's rows stream through once (non-temporal); x is
    // re-read by every block and stays cached. Rows past m read row m - 1 and are dropped.
    constexpr int kUnroll = kRows <= 2 ? 4 : (kRows == 4 ? 2 : 1);
    const long long n4 = n >> 2;
    const f32x4 *__restrict__ x4 = reinterpret_cast<const f32x4 *>(x);
    const f32x4 *a4[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const long long row = min(row0 + r, sld(D.m) - 1);
      a4[r] = reinterpret_cast<const f32x4 *>(A + row * n);
    }
    long long c = threadIdx.x;
    for (; c + (long long)(kUnroll - 1) * kBlock < n4; c += (long long)kUnroll * kBlock) {
      f32x4 xv[kUnroll], av[kRows][kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) xv[u] = x4[c + u * kBlock];
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) av[r][u] = __builtin_nontemporal_load(&a4[r][c + u * kBlock]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int r = 0; r < kRows; ++r)
          acc[r] += av[r][u].x * xv[u].x + av[r][u].y * xv[u].y + av[r][u].z * xv[u].z +
                    av[r][u].w * xv[u].w;
    }
    for (; c < n4; c += kBlock) {
      const f32x4 xv = x4[c];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const f32x4 a = __builtin_nontemporal_load(&a4[r][c]);
        acc[r] += a.x * xv.x + a.y * xv.y + a.z * xv.z + a.w * xv.w;
      }
    }
  } else {
    for (long long c = threadIdx.x; c < n; c += kBlock) {
      const float xv = x[c];
#pragma unroll
      for (int r = 0; r < kRows; ++r)
        if (r < nrows) acc[r] += A[(row0 + r) * n + c] * xv;
    }
  }
  __shared__ float ys[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const float s = block_sum_f(acc[r]);
    if (threadIdx.x == 0) ys[r] = s;
  }
  __syncthreads();
  double dot = 0.0;
  if (threadIdx.x < nrows) {
    const long long i = row0 + threadIdx.x;
    epilogue(D, epi, i, ys[threadIdx.x], nullptr, dot);
  }
  dot = block_sum(dot);
  if (threadIdx.x == 0) sld(D.part)[blockIdx.x] = dot;
}

// Dense adjoint, stage 1: column partial sums over a chunk of rows.
// grid (ceil(n/(4*kBlock)), B, chunks); colpart[chunk][col] = sum_{rows in chunk} A[row][col] u[row]
__global__ void __launch_bounds__(kBlock) k_gemv_cols(InstDesc *const *descs) {
  const InstDesc &D = inst(descs);
  if (stopped_inner(D)) return;
  const long long n = sld(D.n), m = sld(D.m);
  const int chunks = sld(D.colchunks);
  const int ch = blockIdx.z;
  if (ch >= chunks) return;
  const long long rc = (m + chunks - 1) / chunks;
  const long long r0 = ch * rc, r1 = min(m, r0 + rc);
  const float *__restrict__ A = sld(D.A);
  const float *__restrict__ u = sld(D.u);
  float *__restrict__ out = sld(D.colpart) + (long long)ch * n;
  if ((n & 3) == 0) {
    // Rows are taken in order, kRowUnroll at a time with all their loads issued first; u[r] is
    // uniform across the block (scalar loads).
    constexpr int kRowUnroll = 8;
    const long long c4 = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c4 * 4 >= n) return;
    const long long n4 = n >> 2;
    const f32x4 *__restrict__ a4 = reinterpret_cast<const f32x4 *>(A) + c4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    long long r = r0;
    for (; r + kRowUnroll <= r1; r += kRowUnroll) {
      f32x4 av[kRowUnroll];
      float ur[kRowUnroll];
#pragma unroll
      for (int q = 0; q < kRowUnroll; ++q) {
        av[q] = __builtin_nontemporal_load(a4 + (r + q) * n4);
        ur[q] = u[r + q];
      }
#pragma unroll
      for (int q = 0; q < kRowUnroll; ++q) {
        acc.x += av[q].x * ur[q];
        acc.y += av[q].y * ur[q];
        acc.z += av[q].z * ur[q];
        acc.w += av[q].w * ur[q];
      }
    }
    for (; r < r1; ++r) {
      const f32x4 a = __builtin_nontemporal_load(a4 + r * n4);
      const float ur = u[r];
      acc.x += a.x * ur;
      acc.y += a.y * ur;
      acc.z += a.z * ur;
      acc.w += a.w * ur;
    }
    reinterpret_cast<f32x4 *>(out)[c4] = acc;
  } else {
    const long long c0 = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4;
    for (int q = 0; q < 4; ++q) {
      const long long c = c0 + q;
      if (c >= n) break;
      float acc = 0.f;
      for (long long r = r0; r < r1; ++r) acc += A[r * n + c] * u[r];
      out[c] = acc;
    }
  }
}

// Dense adjoint, stage 2: sum the chunk partials and apply the epilogue.
__global__ void __launch_bounds__(kBlock) k_colsum(InstDesc *const *descs, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= sld(D.n)) return;
  float y = 0.f;
  for (int ch = 0; ch < sld(D.colchunks); ++ch) y += sld(D.colpart)[(long long)ch * sld(D.n) + c];
  double dot = 0.0;
  epilogue(D, epi, c, y, nullptr, dot);
}

static inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

#define LAUNCH(kern, gx, gy, ...) \
  hipLaunchKernelGGL(kern, dim3(gx, gy), dim3(kBlock), 0, st, __VA_ARGS__)

int launch_gemv_rows(hipStream_t st, InstDesc *const *d, int B, long long m, int src, int epi,
                     int rows) {
  const unsigned g = (unsigned)((m + rows - 1) / rows);
  switch (rows) {
    case 1: LAUNCH(k_gemv_rows<1>, g, B, d, src, epi); break;
    case 2: LAUNCH(k_gemv_rows<2>, g, B, d, src, epi); break;
    case 8: LAUNCH(k_gemv_rows<8>, g, B, d, src, epi); break;
    default: LAUNCH(k_gemv_rows<4>, g, B, d, src, epi); break;
  }
  return (int)g;
}
void launch_gemv_cols(hipStream_t st, InstDesc *const *d, int B, long long n, int chunks) {
  const unsigned gx = (unsigned)((n + 4 * kBlock - 1) / (4 * kBlock));
  hipLaunchKernelGGL(k_gemv_cols, dim3(gx, B, chunks), dim3(kBlock), 0, st, d);
}
void launch_colsum(hipStream_t st, InstDesc *const *d, int B, long long n, int epi) {
  LAUNCH(k_colsum, blocks_for(n), B, d, epi);
}
}  // namespace plsqr
