// Batched dense products on MFMA for a lockstep batch of instances sharing one dense A.
//
// Forward:  Y (n_Y x Bpad) = A (n_Y x n_X) . X (n_X x Bpad), split over K = n_X.
// Adjoint:  Z (n_X x Bpad) = A^T (n_X x n_Y) . U (n_Y x Bpad), epilogue applied in place.
// Operands are BF16 with FP32 accumulation. Each FP32 operand v is split as
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi); the product keeps hi.hi, hi.lo and
// (optionally) lo.hi terms: the one-step refinement of a single BF16 product.
//
// Tiling (gfx950, v_mfma_f32_32x32x16_bf16, wave64): a block of 8 waves owns 256 rows of
// the left operand; each wave owns 32 rows and all Bpad (= 32 * NT) columns. Per step of
// 128 along K, lane (i, h) (i = lane % 32, h = lane / 32) loads 64 contiguous K values of
// its row (8 x 16-byte loads, prefetched one step ahead) and feeds them to 8 MFMAs; the
// right-operand block of the step (hi and lo, Bpad x 128) is staged once per block in
// LDS (double-buffered, rows padded against bank conflicts) and lane (j, h) reads the
// same 64 K indices of column j, so every MFMA pairs identical K indices (the K order
// inside one 128-step is a permutation, which the sum does not see).
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace plsqr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGemmWaves = 8;                 // waves per block
constexpr int kGemmRows = 32 * kGemmWaves;    // rows of the left operand per block
constexpr int kKStep = 128;                   // K per step
constexpr int kLdsRow = kKStep + 8;           // bf16 per LDS column row (padded: no bank conflicts)

// Right-operand block of one K step in LDS: [hi | lo][Bpad columns][kLdsRow]. Each of
// the 512 threads moves NT * 2 chunks of 16 bytes (held in named registers, not an array,
// so that they never go to scratch).
struct XChunks {
  uint4 v[4];
};

__device__ __forceinline__ void chunk_coords(int q, int NT, int &half, int &col, int &chunk) {
  const int idx = q * 512 + (int)threadIdx.x;   // 16-byte chunk index
  half = idx / (NT * 32 * 16);                   // 0: hi, 1: lo
  const int rem = idx % (NT * 32 * 16);
  col = rem / 16;
  chunk = rem % 16;
}

template <int NT>
__device__ __forceinline__ XChunks stage_right(const __bf16 *__restrict__ Rhi,
                                               const __bf16 *__restrict__ Rlo, long long K,
                                               long long k0) {
  XChunks x;
#pragma unroll
  for (int q = 0; q < NT * 2; ++q) {
    int half, col, chunk;
    chunk_coords(q, NT, half, col, chunk);
    const __bf16 *src = (half ? Rlo : Rhi) + (long long)col * K + k0 + chunk * 8;
    x.v[q] = *reinterpret_cast<const uint4 *>(src);
  }
  return x;
}

template <int NT>
__device__ __forceinline__ void store_right(__bf16 *lds, const XChunks &x) {
#pragma unroll
  for (int q = 0; q < NT * 2; ++q) {
    int half, col, chunk;
    chunk_coords(q, NT, half, col, chunk);
    *reinterpret_cast<uint4 *>(lds + ((half * NT * 32 + col) * kLdsRow + chunk * 8)) = x.v[q];
  }
}

template <int NT, bool LO_L, bool EPI>
__global__ void __launch_bounds__(512, 1) k_gemm_bf16(
    const __bf16 *__restrict__ Lhi, const __bf16 *__restrict__ Llo,
    const __bf16 *__restrict__ Rhi, const __bf16 *__restrict__ Rlo, long long M, long long K,
    long long kchunk, int Bpad, float *__restrict__ out, InstDesc *const *descs, int B, int epi) {
  __shared__ __bf16 lds[2][2 * NT * 32 * kLdsRow];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, h = lane >> 5;
  const long long row0 = (long long)blockIdx.x * kGemmRows + wave * 32;
  const int ks = blockIdx.y;
  const long long kbeg = (long long)ks * kchunk;
  const long long kend = min(K, kbeg + kchunk);
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

  const __bf16 *pa = Lhi + (row0 + li) * K + h * 64;
  const __bf16 *pal = LO_L ? Llo + (row0 + li) * K + h * 64 : nullptr;
  bf16x8 a[8], al[LO_L ? 8 : 1];
  XChunks xr;
  // prologue: step kbeg
  if (kbeg < kend) {
#pragma unroll
    for (int s = 0; s < 8; ++s) a[s] = *reinterpret_cast<const bf16x8 *>(pa + kbeg + s * 8);
    if constexpr (LO_L) {
#pragma unroll
      for (int s = 0; s < 8; ++s) al[s] = *reinterpret_cast<const bf16x8 *>(pal + kbeg + s * 8);
    }
    xr = stage_right<NT>(Rhi, Rlo, K, kbeg);
    store_right<NT>(lds[0], xr);
  }
  __syncthreads();
  int buf = 0;
  for (long long k0 = kbeg; k0 < kend; k0 += kKStep) {
    const long long kn = k0 + kKStep;
    const bool more = kn < kend;
    // prefetch the next step's operands while this step computes
    bf16x8 an[8], aln[LO_L ? 8 : 1];
    if (more) {
#pragma unroll
      for (int s = 0; s < 8; ++s) an[s] = *reinterpret_cast<const bf16x8 *>(pa + kn + s * 8);
      if constexpr (LO_L) {
#pragma unroll
        for (int s = 0; s < 8; ++s) aln[s] = *reinterpret_cast<const bf16x8 *>(pal + kn + s * 8);
      }
      xr = stage_right<NT>(Rhi, Rlo, K, kn);
    }
    const __bf16 *L0 = lds[buf];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = t * 32 + li;
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(L0 + col * kLdsRow + h * 64 + s * 8);
        const bf16x8 bl =
            *reinterpret_cast<const bf16x8 *>(L0 + (NT * 32 + col) * kLdsRow + h * 64 + s * 8);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], b, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], bl, acc[t], 0, 0, 0);
        if constexpr (LO_L)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], b, acc[t], 0, 0, 0);
      }
    }
    if (more) {
      store_right<NT>(lds[buf ^ 1], xr);
#pragma unroll
      for (int s = 0; s < 8; ++s) a[s] = an[s];
      if constexpr (LO_L) {
#pragma unroll
        for (int s = 0; s < 8; ++s) al[s] = aln[s];
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  // accumulator element r of lane (li, h) is (row 8*(r/4) + 4*h + r%4, column li) of the tile
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 32 + li;
    int e = epi;
    bool skip = false;
    if constexpr (EPI) skip = col < B && product_masked(*descs[col], e);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long row = row0 + (r >> 2) * 8 + h * 4 + (r & 3);
      if constexpr (!EPI) {
        out[((long long)ks * M + row) * Bpad + col] = acc[t][r];
      } else {
        if (col < B && !skip) {
          const InstDesc &D = *descs[col];
          double unused = 0.0;
          epilogue(D, e, row, acc[t][r], nullptr, unused);
        }
      }
    }
  }
}

// Sum the forward split-K partials of instance blockIdx.y and apply its epilogue.
__global__ void __launch_bounds__(kBlock) k_fwd_reduce(InstDesc *const *descs, const float *Ypart,
                                                      int ks, long long M, int Bpad, int epi) {
  const InstDesc &D = inst(descs);
  if (product_masked(D, epi)) return;
  const int b = blockIdx.y;
  const long long row = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (row < M) {
    float y = 0.f;
    for (int s = 0; s < ks; ++s) y += Ypart[((long long)s * M + row) * Bpad + b];
    epilogue(D, epi, row, y, nullptr, dot);
  }
  dot = block_sum(dot);
  if (threadIdx.x == 0) D.part[blockIdx.x] = dot;
}

// Pack the right operand: column b of (Rhi, Rlo) = split of vector `sel` of instance b
// (length len); padding columns b >= B are zero.
__global__ void __launch_bounds__(kBlock) k_pack_split(InstDesc *const *descs, int B, int sel,
                                                      long long len, __bf16 *Rhi, __bf16 *Rlo) {
  const int b = blockIdx.y;
  const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (k >= len) return;
  float x = 0.f;
  if (b < B) x = vec_of(*descs[b], sel)[k];
  const __bf16 hi = (__bf16)x;
  const __bf16 lo = (__bf16)(x - (float)hi);
  Rhi[(long long)b * len + k] = hi;
  Rlo[(long long)b * len + k] = lo;
}

// A = hi + lo split of a float32 matrix (elementwise).
__global__ void __launch_bounds__(kBlock) k_split_matrix(const float *A, __bf16 *hi, __bf16 *lo,
                                                        long long count) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < count;
       i += (long long)gridDim.x * kBlock) {
    const float a = A[i];
    const __bf16 h = (__bf16)a;
    hi[i] = h;
    if (lo) lo[i] = (__bf16)(a - (float)h);
  }
}

// out (C x R) = in (R x C)^T for 16-bit elements, 64 x 64 tiles through LDS.
__global__ void __launch_bounds__(kBlock) k_transpose16(const uint16_t *in, uint16_t *out,
                                                       long long R, long long C) {
  __shared__ uint16_t tile[64][65];
  const long long c0 = (long long)blockIdx.x * 64, r0 = (long long)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
  for (int i = ty; i < 64; i += 4) {
    const long long r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < R && c < C) ? in[r * C + c] : (uint16_t)0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const long long c = c0 + i, r = r0 + tx;
    if (c < C && r < R) out[c * R + r] = tile[tx][i];
  }
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
template <int NT, bool LO_L, bool EPI>
static void gemm_launch(hipStream_t st, const void *Lhi, const void *Llo, const void *Rhi,
                        const void *Rlo, long long M, long long K, long long kchunk, int ks,
                        int Bpad, float *out, InstDesc *const *descs, int B, int epi) {
  hipLaunchKernelGGL((k_gemm_bf16<NT, LO_L, EPI>), dim3((unsigned)(M / kGemmRows), ks),
                     dim3(64 * kGemmWaves), 0, st, (const __bf16 *)Lhi, (const __bf16 *)Llo,
                     (const __bf16 *)Rhi, (const __bf16 *)Rlo, M, K, kchunk, Bpad, out, descs, B,
                     epi);
}

template <bool EPI>
static void gemm_dispatch(hipStream_t st, int NT, bool lo_l, const void *Lhi, const void *Llo,
                          const void *Rhi, const void *Rlo, long long M, long long K,
                          long long kchunk, int ks, int Bpad, float *out, InstDesc *const *descs,
                          int B, int epi) {
  if (NT == 1) {
    if (lo_l) gemm_launch<1, true, EPI>(st, Lhi, Llo, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
    else gemm_launch<1, false, EPI>(st, Lhi, Llo, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
  } else {
    if (lo_l) gemm_launch<2, true, EPI>(st, Lhi, Llo, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
    else gemm_launch<2, false, EPI>(st, Lhi, Llo, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
  }
}

// Forward product of the batch: u-epilogue (or residual) per instance; returns partials.
int launch_gemm_forward(hipStream_t st, InstDesc *const *d, int B, const GemmArgs &g, long long m,
                        long long n, int src_sel, int epi) {
  const unsigned pb = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_split, dim3(pb, g.Bpad), dim3(kBlock), 0, st, d, B, src_sel, n,
                     (__bf16 *)g.X_hi, (__bf16 *)g.X_lo);
  gemm_dispatch<false>(st, g.Bpad / 32, g.use_A_lo != 0, g.A_hi, g.A_lo, g.X_hi, g.X_lo, m, n,
                       g.kchunk, g.ks, g.Bpad, g.Ypart, d, B, epi);
  const unsigned rb = (unsigned)((m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_fwd_reduce, dim3(rb, B), dim3(kBlock), 0, st, d, (const float *)g.Ypart, g.ks,
                     m, g.Bpad, epi);
  return (int)rb;
}

// Adjoint product of the batch with the p-epilogue applied in the GEMM.
void launch_gemm_adjoint(hipStream_t st, InstDesc *const *d, int B, const GemmArgs &g, long long m,
                         long long n, int epi) {
  const unsigned pb = (unsigned)((m + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_split, dim3(pb, g.Bpad), dim3(kBlock), 0, st, d, B, (int)V_U, m,
                     (__bf16 *)g.U_hi, (__bf16 *)g.U_lo);
  gemm_dispatch<true>(st, g.Bpad / 32, g.use_A_lo != 0, g.At_hi, g.At_lo, g.U_hi, g.U_lo, n, m, m,
                      1, g.Bpad, nullptr, d, B, epi);
}

void launch_split_matrix(hipStream_t st, const float *A, void *hi, void *lo, long long count) {
  hipLaunchKernelGGL(k_split_matrix, dim3(8192), dim3(kBlock), 0, st, A, (__bf16 *)hi, (__bf16 *)lo,
                     count);
}

void launch_transpose16(hipStream_t st, const void *in, void *out, long long R, long long C) {
  hipLaunchKernelGGL(k_transpose16, dim3((unsigned)((C + 63) / 64), (unsigned)((R + 63) / 64)),
                     dim3(kBlock), 0, st, (const uint16_t *)in, (uint16_t *)out, R, C);
}

}  // namespace plsqr
