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
// 64 along K, lane (i, h) (i = lane % 32, h = lane / 32) loads 32 contiguous K values of
// its row (4 x 16-byte loads per part, issued three steps ahead) and feeds them to 4 MFMAs.
// The left operand is stored tiled (the library builds it once per operator, see
// k_split_tiled): each 32-row x 64-K tile of one part is 4 KB contiguous with lane (i, h)'s
// 16-byte vector for load s at vector index s * 64 + lane, and the hi tile is followed by the
// lo tile of the same rows and K range. In the forward operand the 8 KB tile pairs of the 8
// row tiles of one block (256 rows) at one K step are adjacent and the K steps follow each
// other, so a block streams one 64 KB run per step; in the adjoint operand each row tile's
// pairs follow each other along K, so each wave streams its own 8 KB per step (measured on the
// 8192 x 262144 batch: the forward product, one round of 256 blocks, is 4% faster grouped; the
// adjoint, four rounds of 256, 4% slower). Each load instruction of a wave reads 1 KB
// contiguous (a row-major operand would make every load instruction gather 16 bytes from 32
// rows 2 K apart, re-requesting each cache line 8 times and scattering DRAM accesses over all
// rows of the tile; separate hi and lo arrays would give each wave two streams 4 GiB apart);
// the
// right-operand block of the step (hi and lo, Bpad x 64) is staged once per block in
// LDS (double-buffered, rows padded against bank conflicts) and lane (j, h) reads the
// same 32 K indices of column j, so every MFMA pairs identical K indices (the K order
// inside one 64-step is a permutation, which the sum does not see).
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace plsqr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kGemmWaves = 8;                 // waves per block
constexpr int kGemmRows = 32 * kGemmWaves;    // rows of the left operand per block
constexpr int kKStep = 64;                    // K per step
constexpr int kSlots = kKStep / 16;           // MFMAs along K per step (8 K per lane half)
constexpr int kLdsRow = kKStep + 8;           // bf16 per LDS column row (padded: no bank conflicts)
constexpr int kTileElems = 32 * kKStep;       // elements of one 32-row x 64-K left-operand tile
constexpr int kPairElems = 2 * kTileElems;    // a hi tile and its lo tile
constexpr int kGroupFwd = kGemmWaves;         // row tiles whose pairs interleave per K step:
constexpr int kGroupAdj = 1;                  // forward operand, adjoint operand
constexpr int kChunks = kKStep / 8;           // 16-byte chunks of one column per step

// Right-operand block of one K step in LDS: [hi | lo][Bpad columns][kLdsRow]. Each of
// the 512 threads moves NT * kKStep / 64 chunks of 16 bytes (held in named registers, not an
// array, so that they never go to scratch).
struct XChunks {
  uint4 v[2];
};

__device__ __forceinline__ void chunk_coords(int q, int NT, int &half, int &col, int &chunk) {
  const int idx = q * 512 + (int)threadIdx.x;   // 16-byte chunk index
  half = idx / (NT * 32 * kChunks);              // 0: hi, 1: lo
  const int rem = idx % (NT * 32 * kChunks);
  col = rem / kChunks;
  chunk = rem % kChunks;
}

template <int NT>
__device__ __forceinline__ XChunks stage_right(const __bf16 *__restrict__ Rhi,
                                               const __bf16 *__restrict__ Rlo, long long K,
                                               long long k0) {
  XChunks x;
#pragma unroll
  for (int q = 0; q < NT * kKStep / 64; ++q) {
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
  for (int q = 0; q < NT * kKStep / 64; ++q) {
    int half, col, chunk;
    chunk_coords(q, NT, half, col, chunk);
    *reinterpret_cast<uint4 *>(lds + ((half * NT * 32 + col) * kLdsRow + chunk * 8)) = x.v[q];
  }
}

template <int NT, bool LO_L, bool EPI>
__global__ void __launch_bounds__(512, 1) k_gemm_bf16(
    const __bf16 *__restrict__ L, const __bf16 *__restrict__ Rhi, const __bf16 *__restrict__ Rlo, long long M, long long K,
    long long kchunk, int group, int Bpad, float *__restrict__ out, InstDesc *const *descs, int B,
    int epi) {
  __shared__ __bf16 lds[2][2 * NT * 32 * kLdsRow];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, h = lane >> 5;
  // (row group, K split) of this block: workgroups are dealt to the 8 XCDs round-robin in
  // linear order, so taking the split from the low part of the linear index puts the blocks of
  // one split on one XCD (with 8 splits), whose L2 then serves that split's right operand
  const long long bid = (long long)blockIdx.y * gridDim.x + blockIdx.x;
  const long long rgrp = bid / gridDim.y;
  const int ks = (int)(bid % gridDim.y);
  const long long row0 = rgrp * kGemmRows + wave * 32;
  const long long kbeg = (long long)ks * kchunk;
  const long long kend = min(K, kbeg + kchunk);
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

  // this wave's row tile rt in the tiled operand: step st is pair
  // (rt / group * K/64 + kbeg / kKStep + st) * group + rt % group, load s of lane `lane` is
  // vector s * 64 + lane of the pair's hi and lo tiles
  const long long rt = row0 / 32;
  const long long pair0 = ((rt / group) * (K / kKStep) + kbeg / kKStep) * group + rt % group;
  // loads issued past the last step read the first 4 KB of the right operand instead (valid,
  // cached, never used): re-reading the left operand would fetch it from memory again
  const __bf16 *pa = L + pair0 * kPairElems + lane * 8;
  const __bf16 *pal = pa + kTileElems;
  const long long step_elems = (long long)group * kPairElems;
  const long long nsteps = (kend - kbeg) / kKStep;   // kchunk and K are multiples of kKStep
  // Pipeline: the left operand of step st + 3 and the right operand of step st + 2 are
  // issued while step st computes, in that order of issue per step (right, then left), so
  // that every wait retires only loads that are due: the right operand of step st + 1 is
  // awaited at the end of step st (it was issued before the left operand of step st + 2),
  // the left operand of step st + 1 at the start of step st + 1. Left operands rotate through
  // four register sets, right operands through two, the LDS copy of the right operand through
  // two buffers.
  struct AStep {
    bf16x8 hi[kSlots], lo[LO_L ? kSlots : 1];
  };
  // loads past the last step are redirected (a select, not a branch): the loop body has no
  // branches, so the compiler's wait counts follow the order of issue exactly
  // the left operand is read exactly once: non-temporal loads stream it past the caches,
  // which keep the right operand that every row block re-reads
  auto ld_nt = [](const __bf16 *p) {
    return __builtin_bit_cast(bf16x8, __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p)));
  };
  auto load_a = [&](AStep &a, long long st) {
    const bool in = st < nsteps;
    const __bf16 *ph = in ? pa + st * step_elems : Rhi + lane * 8;
    const __bf16 *pl = in ? pal + st * step_elems : Rhi + lane * 8;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) a.hi[q] = ld_nt(ph + q * 512);
    if constexpr (LO_L) {
#pragma unroll
      for (int q = 0; q < kSlots; ++q) a.lo[q] = ld_nt(pl + q * 512);
    }
  };
  auto load_x = [&](XChunks &x, long long st) {
    x = stage_right<NT>(Rhi, Rlo, K, kbeg + min(st, nsteps - 1) * kKStep);
  };
  AStep a0, a1, a2, a3;
  XChunks x0, x1;
  // (scheduling barriers keep the loads in this order of issue: the waits below rely on it;
  // the host plans every block's K range as a positive multiple of 4 steps)
  {
    XChunks xf;
    load_x(xf, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_x(x1, 1);
    __builtin_amdgcn_sched_barrier(0);
    load_a(a0, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(a1, 1);
    __builtin_amdgcn_sched_barrier(0);
    load_a(a2, 2);
    __builtin_amdgcn_sched_barrier(0);
    store_right<NT>(lds[0], xf);
  }
  __syncthreads();
  // step st computes with left set `cur` and LDS buffer st % 2; it issues the right operand of
  // step st + 2 into `xn` and the left operand of step st + 3 into `an` (both free now), then
  // stores the right operand of step st + 1 (held in `xs`) into LDS buffer (st + 1) % 2.
  auto step = [&](const AStep &cur, AStep &an, XChunks &xn, const XChunks &xs, long long st) {
    load_x(xn, st + 2);
    __builtin_amdgcn_sched_barrier(0);
    load_a(an, st + 3);
    __builtin_amdgcn_sched_barrier(0);
    const __bf16 *L0 = lds[st & 1];
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = t * 32 + li;
        const int ko = h * (kKStep / 2) + q * 8;
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(L0 + col * kLdsRow + ko);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(L0 + (NT * 32 + col) * kLdsRow + ko);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur.hi[q], b, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur.hi[q], bl, acc[t], 0, 0, 0);
        if constexpr (LO_L)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur.lo[q], b, acc[t], 0, 0, 0);
      }
    }
    store_right<NT>(lds[(st + 1) & 1], xs);   // past the last step: unused, harmless
    __syncthreads();
  };
  // four steps per trip: the register sets rotate with period 4 (left) and 2 (right)
  for (long long st = 0; st < nsteps; st += 4) {
    step(a0, a3, x0, x1, st);
    step(a1, a0, x1, x0, st + 1);
    step(a2, a1, x0, x1, st + 2);
    step(a3, a2, x1, x0, st + 3);
  }
  // accumulator element r of lane (li, h) is (row 8*(r/4) + 4*h + r%4, column li) of the tile
  auto row_of = [&](int r) { return row0 + (r >> 2) * 8 + h * 4 + (r & 3); };
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 32 + li;
    if constexpr (!EPI) {
#pragma unroll
      for (int r = 0; r < 16; ++r) out[((long long)ks * M + row_of(r)) * Bpad + col] = acc[t][r];
    } else {
      // The adjoint epilogue of instance `col` on this lane's 16 rows (EPI_ADJ_INIT: p = su y;
      // EPI_ADJ: p = su y - (beta sv) p, the only codes this kernel is launched with). The
      // instance's scalars are read once and the 16 old values of p are loaded before any is
      // stored, so the lane waits on memory once rather than once per row.
      int e = epi;
      if (col < B && !product_masked(*descs[col], e)) {
        const InstDesc &D = *descs[col];
        float *p = sld(D.p);
        const double *sc = sld(D.sc);
        const float c1 = (float)sc[SC_SU];
        const bool upd = (e == EPI_ADJ);
        const float c2 = upd ? (float)(sc[SC_BETA] * sc[SC_SV]) : 0.f;
        float old[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) old[r] = upd ? p[row_of(r)] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) p[row_of(r)] = upd ? c1 * acc[t][r] - c2 * old[r] : c1 * acc[t][r];
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
// (length len); padding columns b >= B are zero. upd (forward product from v): also apply the
// instance's pending f, w update (SC_UPD: f += (phi/rho) w, w = v / alpha - (theta/rho) w, the
// arithmetic of k_update_fw) to element k, which this thread reads anyway.
__global__ void __launch_bounds__(kBlock) k_pack_split(InstDesc *const *descs, int B, int sel,
                                                      long long len, __bf16 *Rhi, __bf16 *Rlo,
                                                      int upd) {
  const int b = blockIdx.y;
  const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (k >= len) return;
  float x = 0.f;
  if (b < B) {
    const InstDesc &D = *descs[b];
    x = vec_of(D, sel)[k];
    const double *sc = sld(D.sc);
    if (upd && sc[SC_UPD] != 0.0 && sc[SC_STOP] == 0.0) {
      const float cf = (float)sc[SC_CF], cw = (float)sc[SC_CW], sv = (float)sc[SC_SV];
      float *f = sld(D.f), *w = sld(D.w);
      const float wk = w[k];
      f[k] += cf * wk;
      w[k] = sv * x - cw * wk;
    }
  }
  const __bf16 hi = (__bf16)x;
  const __bf16 lo = (__bf16)(x - (float)hi);
  Rhi[(long long)b * len + k] = hi;
  Rlo[(long long)b * len + k] = lo;
}

// Tiled left operands (layout described at the top of this file). Vector v (16 bytes, 8
// elements) of one part of the tiled M x K operand L is vector s * 64 + lane of tile (rt, kt),
// with v = ((rt * K/64 + kt) * 4 + s) * 64 + lane; it holds L[row][k0 .. k0 + 7] with
// row = 32 rt + lane % 32 and k0 = 64 kt + 32 (lane / 32) + 8 s. It sits at element
// pair_offset(v, K, group) of the hi/lo pair array (hi part), kTileElems further on (lo part):
// tile (rt, kt) is pair (rt / group * K/64 + kt) * group + rt % group. L is A (n_y x n_x) for
// the forward product (transposed = 0, group kGroupFwd) or A^T for the adjoint
// (transposed = 1, group kGroupAdj).
__device__ __forceinline__ void tiled_coords(long long v, long long K, int transposed,
                                             long long n_x, long long &row, long long &k0,
                                             long long &stride) {
  const int lane = (int)(v % 64);
  const long long q = v / 64;
  const int s = (int)(q % kSlots);
  const long long tile = q / kSlots;
  const long long nkt = K / kKStep;
  row = (tile / nkt) * 32 + (lane & 31);
  k0 = (tile % nkt) * kKStep + (lane >> 5) * (kKStep / 2) + s * 8;
  stride = transposed ? n_x : 1;     // distance between L[row][k] and L[row][k + 1] in A
}

__device__ __forceinline__ long long pair_offset(long long v, long long K, int group) {
  constexpr int kTileVecs = kTileElems / 8;
  const long long tile = v / kTileVecs, nkt = K / kKStep;
  const long long rt = tile / nkt, kt = tile % nkt;
  const long long pair = ((rt / group) * nkt + kt) * group + rt % group;
  return pair * kPairElems + (v % kTileVecs) * 8;
}

// hi = bf16(L), lo = bf16(L - hi) in the tiled pair layout, from the float32 row-major A.
__global__ void __launch_bounds__(kBlock) k_split_tiled(const float *A, long long n_y,
                                                       long long n_x, int transposed,
                                                       __bf16 *dst) {
  const long long M = transposed ? n_x : n_y, K = transposed ? n_y : n_x;
  const long long nvec = M * K / 8;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < nvec;
       v += (long long)gridDim.x * kBlock) {
    long long row, k0, stride;
    tiled_coords(v, K, transposed, n_x, row, k0, stride);
    const float *src = transposed ? A + k0 * n_x + row : A + row * n_x + k0;
    bf16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float a = src[e * stride];
      h[e] = (__bf16)a;
      l[e] = (__bf16)(a - (float)h[e]);
    }
    __bf16 *o = dst + pair_offset(v, K, transposed ? kGroupAdj : kGroupFwd);
    *reinterpret_cast<bf16x8 *>(o) = h;
    *reinterpret_cast<bf16x8 *>(o + kTileElems) = l;
  }
}

// The tiled layout of a 16-bit row-major copy of A (n_y x n_x), as L = A or L = A^T, into
// part `part` (0: hi, 1: lo) of the tile pairs.
__global__ void __launch_bounds__(kBlock) k_retile16(const uint16_t *src16, long long n_y,
                                                    long long n_x, int transposed, int part,
                                                    uint16_t *dst) {
  const long long M = transposed ? n_x : n_y, K = transposed ? n_y : n_x;
  const long long nvec = M * K / 8;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < nvec;
       v += (long long)gridDim.x * kBlock) {
    long long row, k0, stride;
    tiled_coords(v, K, transposed, n_x, row, k0, stride);
    const uint16_t *src = transposed ? src16 + k0 * n_x + row : src16 + row * n_x + k0;
    uint16_t w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = src[e * stride];
    *reinterpret_cast<uint4 *>(dst + pair_offset(v, K, transposed ? kGroupAdj : kGroupFwd) +
                               part * kTileElems) =
        make_uint4(w[0] | ((uint32_t)w[1] << 16), w[2] | ((uint32_t)w[3] << 16),
                   w[4] | ((uint32_t)w[5] << 16), w[6] | ((uint32_t)w[7] << 16));
  }
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
template <int NT, bool LO_L, bool EPI>
static void gemm_launch(hipStream_t st, const void *L, const void *Rhi, const void *Rlo,
                        long long M, long long K, long long kchunk, int ks, int Bpad, float *out,
                        InstDesc *const *descs, int B, int epi) {
  // the epilogue variant is the adjoint product, whose operand is tiled with kGroupAdj
  hipLaunchKernelGGL((k_gemm_bf16<NT, LO_L, EPI>), dim3((unsigned)(M / kGemmRows), ks),
                     dim3(64 * kGemmWaves), 0, st, (const __bf16 *)L, (const __bf16 *)Rhi,
                     (const __bf16 *)Rlo, M, K, kchunk, EPI ? kGroupAdj : kGroupFwd, Bpad, out,
                     descs, B, epi);
}

template <bool EPI>
static void gemm_dispatch(hipStream_t st, int NT, bool lo_l, const void *L, const void *Rhi,
                          const void *Rlo, long long M, long long K, long long kchunk, int ks,
                          int Bpad, float *out, InstDesc *const *descs, int B, int epi) {
  if (NT == 1) {
    if (lo_l) gemm_launch<1, true, EPI>(st, L, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
    else gemm_launch<1, false, EPI>(st, L, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
  } else {
    if (lo_l) gemm_launch<2, true, EPI>(st, L, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
    else gemm_launch<2, false, EPI>(st, L, Rhi, Rlo, M, K, kchunk, ks, Bpad, out, descs, B, epi);
  }
}

// Forward product of the batch: u-epilogue (or residual) per instance; returns partials.
int launch_gemm_forward(hipStream_t st, InstDesc *const *d, int B, const GemmArgs &g, long long m,
                        long long n, int src_sel, int epi, int upd) {
  const unsigned pb = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_split, dim3(pb, g.Bpad), dim3(kBlock), 0, st, d, B, src_sel, n,
                     (__bf16 *)g.X_hi, (__bf16 *)g.X_lo, upd);
  gemm_dispatch<false>(st, g.Bpad / 32, g.use_A_lo != 0, g.A_t, g.X_hi, g.X_lo, m, n, g.kchunk,
                       g.ks, g.Bpad, g.Ypart, d, B, epi);
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
                     (__bf16 *)g.U_hi, (__bf16 *)g.U_lo, 0);
  gemm_dispatch<true>(st, g.Bpad / 32, g.use_A_lo != 0, g.At_t, g.U_hi, g.U_lo, n, m, m, 1,
                      g.Bpad, nullptr, d, B, epi);
}

void launch_split_tiled(hipStream_t st, const float *A, long long n_y, long long n_x,
                        int transposed, void *dst) {
  hipLaunchKernelGGL(k_split_tiled, dim3(8192), dim3(kBlock), 0, st, A, n_y, n_x, transposed,
                     (__bf16 *)dst);
}

void launch_retile16(hipStream_t st, const void *src, long long n_y, long long n_x,
                     int transposed, int part, void *dst) {
  hipLaunchKernelGGL(k_retile16, dim3(8192), dim3(kBlock), 0, st, (const uint16_t *)src, n_y, n_x,
                     transposed, part, (uint16_t *)dst);
}

}  // namespace plsqr
