// The scalar steps of Algorithm 2 that follow a reduction (the square roots giving beta and
// alpha, the damped and plain Givens rotations of (3.6), the per-outer records): one thread
// applies them to an instance's scalar block once the partial sums of a launch are added up.
// They run either in a one-block launch of their own (k_finalize) or in a finaliser block that
// rides along in the next launch (the first pass of a blur product, which reads no scalar that
// the finaliser writes), with the same sum and the same arithmetic.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace plsqr {

// The finaliser's sum of an instance's nparts partials (valid in thread 0), for a block of any
// multiple of 64 threads: it adds exactly as block_sum over kBlock threads would, each of which
// first adds the strided subset v, v + kBlock, ... in order -- virtual thread v's sum is formed
// by thread v mod blockDim.x --, then wave 0 reduces the kBlock / 64 virtual waves one after the
// other with block_sum's shuffle tree and adds their sums in order. The partials come from an
// earlier launch.
__device__ __forceinline__ double parts_sum(const double *part, int nparts) {
  __shared__ double vsum[kBlock];
  for (int v = threadIdx.x; v < kBlock; v += blockDim.x) {
    double s = 0.0;
    for (int i = v; i < nparts; i += kBlock) s += part[i];
    vsum[v] = s;
  }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < 64) {
    for (int w = 0; w < kBlock / 64; ++w) {
      double s = vsum[64 * w + threadIdx.x];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
      r += s;
    }
  }
  return r;
}

// Thread 0: the recurrences of finaliser `what` (Fin) on the summed partials s.
__device__ __forceinline__ void fin_apply(const InstDesc &D, double s, int what) {
  double *sc = sld(D.sc);
  const int k = (int)sc[SC_OUTER];
  double *dg = sld(D.diag) + (long long)k * DG_COUNT;
  auto fail = [&](int code) {
    if (sc[SC_STATUS] == 0.0) sc[SC_STATUS] = (double)code;
    sc[SC_STOP] = 1.0;
  };
  bool keep_upd = false;
  if (what == FIN_ALPHA_PEND || what == FIN_ALPHA_PEND_T) {
    if (what == FIN_ALPHA_PEND_T) sc[SC_UPD] = 0.0;   // the last V-cycle's tail applied it
    if (sc[SC_FINA] == 0.0) return;
    sc[SC_FINA] = 0.0;
    what = FIN_ALPHA;
  } else if (what == FIN_BETA_PEND || what == FIN_BETA_PEND_T) {
    sc[SC_FINA] = 1.0;   // the V-cycle after this product leaves its partials for FIN_ALPHA_PEND
    keep_upd = (what == FIN_BETA_PEND_T);   // the update waits for that V-cycle's tail
    what = FIN_BETA;
  }
  switch (what) {
    case FIN_BETA_INIT: {
      sc[SC_UPD] = 0.0;
      if (sc[SC_HALT] != 0.0) break;   // the partials were not written (outer loop ended)
      const double beta = sqrt(s);
      if (!isfinite(beta)) { fail(PLSQR_E_NONFINITE); break; }
      if (beta <= kTiny) { sc[SC_STOP] = 1.0; break; }
      sc[SC_BETA] = beta;
      sc[SC_SU] = 1.0 / beta;
      sc[SC_PHIBAR] = beta;
      if (double *h = sld(D.hist)) h[sld(D.inner_count) + 1] = beta;   // beta_1
      break;
    }
    case FIN_ALPHA_INIT: {
      sc[SC_UPD] = 0.0;
      sc[SC_FINA] = 0.0;
      if (sc[SC_STOP] != 0.0) break;
      if (!isfinite(s)) { fail(PLSQR_E_NONFINITE); break; }
      if (s < 0.0) { fail(PLSQR_E_NOT_SPD); break; }
      const double alpha = sqrt(s);
      if (alpha <= kTiny) { sc[SC_STOP] = 1.0; break; }
      sc[SC_ALPHA] = alpha;
      sc[SC_SV] = 1.0 / alpha;
      sc[SC_RHOBAR] = alpha;
      if (double *h = sld(D.hist)) h[0] = alpha;   // alpha_1
      break;
    }
    case FIN_BETA: {
      // the forward product that precedes this applied any pending update (unless it waits for
      // the V-cycle's tail)
      if (!keep_upd) sc[SC_UPD] = 0.0;
      if (sc[SC_STOP] != 0.0) break;
      const double beta = sqrt(s);
      if (!isfinite(beta)) { fail(PLSQR_E_NONFINITE); break; }
      if (beta <= kTiny) { sc[SC_STOP] = 1.0; break; }
      sc[SC_BETA] = beta;
      sc[SC_SU] = 1.0 / beta;
      // beta_{i+1} of step i (SC_DONE = i - 1 steps completed so far)
      if (double *h = sld(D.hist)) {
        const int i = (int)sc[SC_DONE] + 1;
        if (i <= sld(D.inner_count)) h[sld(D.inner_count) + 1 + i] = beta;
      }
      break;
    }
    case FIN_ALPHA: {
      if (sc[SC_STOP] != 0.0) break;
      if (!isfinite(s)) { fail(PLSQR_E_NONFINITE); break; }
      if (s < 0.0) { fail(PLSQR_E_NOT_SPD); break; }
      const double alpha = sqrt(s);
      if (alpha <= kTiny) { sc[SC_STOP] = 1.0; break; }
      const double beta = sc[SC_BETA], lam = sc[SC_LAMBDA];
      double rhobar = sc[SC_RHOBAR], phibar = sc[SC_PHIBAR];
      if (double *h = sld(D.hist)) {   // alpha_{i+1} of step i
        const int i = (int)sc[SC_DONE] + 1;
        if (i <= sld(D.inner_count)) h[i] = alpha;
      }
      // damping rotation (row sqrt(tau) of (3.6)), then the Givens rotation with beta
      const double rhohat = hypot(rhobar, lam);
      const double c1 = rhobar / rhohat;
      phibar = c1 * phibar;
      const double rho = hypot(rhohat, beta);
      const double c = rhohat / rho, sn = beta / rho;
      const double theta = sn * alpha;
      rhobar = -c * alpha;
      const double phi = c * phibar;
      phibar = sn * phibar;
      sc[SC_CF] = phi / rho;
      sc[SC_CW] = theta / rho;
      sc[SC_RHOBAR] = rhobar;
      sc[SC_PHIBAR] = phibar;
      sc[SC_ALPHA] = alpha;
      sc[SC_SV] = 1.0 / alpha;
      sc[SC_DONE] += 1.0;
      sc[SC_UPD] = 1.0;
      break;
    }
    case FIN_RESID: {
      sc[SC_UPD] = 0.0;
      if (sc[SC_HALT] != 0.0) break;
      dg[DG_RESID] = sqrt(s);
      dg[DG_INNER] = sc[SC_DONE];
      dg[DG_STATUS] = sc[SC_STATUS];
      break;
    }
    case FIN_PENALTY: {
      if (sc[SC_HALT] != 0.0) break;
      dg[DG_PENALTY] = s;
      // outer stop (Algorithm 3, step 5): R(f^k) no longer falls by more than outer_rtol
      if ((sld(D.stop_flags) & PLSQR_FLAG_STOP_OUTER) && k >= sld(D.outer_min)) {
        const double prev = dg[-DG_COUNT + DG_PENALTY];
        if (s - prev >= -sld(D.outer_rtol) * prev) {
          sc[SC_HALT] = 1.0;
          sc[SC_STOP] = 1.0;
        }
      }
      break;
    }
    case FIN_S4: {
      // discrepancy principle S4 on the iterate of the step just completed
      if (sc[SC_STOP] != 0.0) break;
      const double r = sqrt(s);
      sc[SC_S4R] = r;
      if (!isfinite(r)) { fail(PLSQR_E_NONFINITE); break; }
      if (r <= sld(D.s4_level)) sc[SC_STOP] = 1.0;
      break;
    }
    default: break;
  }
}

// The finaliser block of a launch (all its threads): finaliser `what` of instance D on its
// nparts partials, written by an earlier launch.
__device__ __forceinline__ void fin_block(const InstDesc &D, int nparts, int what) {
  const double s = parts_sum(sld(D.part), nparts);
  if (threadIdx.x == 0) fin_apply(D, s, what);
}

}  // namespace plsqr
