// Host-side launchers of the batched HIP kernels. Each takes the stream, a device array
// of B instance-descriptor pointers and the largest extent among the B instances; the
// ones that reduce return the number of partials written per instance.
#pragma once
#include <hip/hip_runtime_api.h>

#include "plsqr_internal.hpp"

namespace plsqr {

// level buffer selectors
enum LevelBuf : int { LB_X = 0, LB_B, LB_R, LB_T, LB_S };

// One-workgroup V-cycle tail: threads, and the largest level it takes over.
constexpr int kTailBlock = 1024;
constexpr long long kTailCells = 4096;
// LDS-resident tail: floats of its pool (eight arrays per level: 16^3 + 8^3 + 4^3 fit)
constexpr int kTailLdsFloats = 37888;
// most cells per thread on a level of the LDS-resident tail (kTailBlock threads)
constexpr int kTailMaxPer = 4;
// highest Chebyshev smoother degree a problem may ask for
constexpr int kMaxChebDegree = 16;

void launch_request_begin(hipStream_t st, InstDesc *const *d, int B, long long n);
void launch_outer_begin(hipStream_t st, InstDesc *const *d, int B);
int launch_diffusivity(hipStream_t st, InstDesc *const *d, int B, long long n, int write_kappa);
void launch_level0_dinv(hipStream_t st, InstDesc *const *d, int B, long long n);
void launch_coarsen(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse);
void launch_level_dinv(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l);
void launch_coarse_factor(hipStream_t st, InstDesc *const *d, int B);
void launch_coarse_solve(hipStream_t st, InstDesc *const *d, int B);
int launch_jacobi(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int first,
                  int src, int dst, int want_dot);
void launch_cheb_start(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int zero_x,
                       int d_sel);
int launch_cheb_step(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int set_x,
                     int update_r, int last, int d_sel, int dn_sel, int step, int want_dot,
                     int add_prolong = 0);
int launch_jacobi_first2(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int dst,
                         int want_dot);
int launch_jacobi_prolong(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int src,
                          int dst, int want_dot);
void launch_cheb_first(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int last,
                       int dn_sel);
void launch_cheb_start_prolong(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l,
                               int d_sel);
void launch_restrict_fine(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse,
                          int nchild, int x_sel, int use_r);
// four-voxel-per-thread forms of the level kernels (smooth_vec.hip): the level's nx must be a
// multiple of 4
int launch_jacobi4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int first,
                   int src, int dst, int want_dot);
int launch_jacobi_first2_4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int dst,
                           int want_dot);
int launch_jacobi_prolong4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int src,
                           int dst, int want_dot);
void launch_cheb_first4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int last,
                        int dn_sel);
void launch_cheb_start_prolong4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l,
                                int d_sel);
void launch_cheb_start4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int zero_x,
                        int d_sel);
int launch_cheb_step4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_l, int set_x,
                      int update_r, int last, int d_sel, int dn_sel, int step, int want_dot,
                      int add_prolong);
void launch_restrict4(hipStream_t st, InstDesc *const *d, int B, int l, long long n_coarse,
                      int x_sel, int use_r);
// levels t .. coarsest of a V-cycle in one workgroup per instance (t >= 1; levels t .. L-2 with
// nx % 4 == 0)
void launch_vcycle_tail(hipStream_t st, InstDesc *const *d, int B, int t);
// the same with every tail level resident in LDS (tail_lds.hip); the levels t .. coarsest must
// need at most kTailLdsFloats floats: tail_lds_floats of their cell counts. t < 0: each
// instance's own first tail level (its descriptor's tail_lds_t). upd_parts > 0: the launch also
// applies each instance's pending f, w update (SC_UPD; n % 4 == 0) in upd_parts more workgroups
// per instance.
void launch_vcycle_tail_lds(hipStream_t st, InstDesc *const *d, int B, int t, int upd_parts = 0);
long long tail_lds_floats(const long long *cells, int nlev);
// Fused level kernels (zmarch.hip): one launch per level and V-cycle half. ZM_*_DOWN runs the
// whole pre-smoothing of level l from x = 0 on b_l, writes the pre-smoothed iterate to the
// level's t buffer and the restricted residual to b_{l+1}; ZM_*_UP adds the coarse correction
// x_{l+1} to that iterate, runs the whole post-smoothing and writes x_l (v on level 0; with
// want_dot the partials of v.p, one per block). H: Jacobi sweeps, or the Chebyshev degree
// (one polynomial per side); the level's nx must be a multiple of 4.
enum ZmKind : int { ZM_JAC_DOWN = 0, ZM_JAC_UP, ZM_CHEB_DOWN, ZM_CHEB_UP };
struct ZmShape {
  int tx, ty, zc;   // output tile: tx x-columns (a multiple of v), ty rows, zc planes
  int v;            // voxels per thread: 4 (x-consecutive) or 1
};
// Default tile for a level of nx x ny x nz (knobs > 0 override ty, zc and v).
ZmShape zm_shape(int nx, int ny, int nz, int H, int ty_knob, int zc_knob, int v_knob);
bool zm_fits(int nx, int H, const ZmShape &s);
long long zm_tiles(int nx, int ny, int nz, const ZmShape &s);   // blocks per instance
size_t zm_lds_bytes(int H, const ZmShape &s, bool down);
int launch_zm(hipStream_t st, InstDesc *const *d, int B, int kind, int H, int l, int nx, int ny,
              int nz, const ZmShape &s, int want_dot);
// The same over a ragged map (each instance's level-l tile from its descriptor's zmp[l], all of
// them with s.v voxels per thread); threads and LDS: the largest over the instances.
void launch_zm_ragged(hipStream_t st, InstDesc *const *d, int kind, int H, int l, int v,
                      int threads, size_t lds, const Rag &rg, int want_dot);
int zm_threads(const ZmShape &s, int H);
// separable blur passes (blur.hip); the x pass takes 16-byte windows when nx % 4 == 0
// groups: 4-output groups per thread when nx % 4 == 0 (1, 2 or 4; 0: default)
// rg: a ragged map (then nx % 4 == 0 for every instance), or kNoRag for B same-shaped
// instances; returns the blocks per instance of a uniform launch
// upd: the first pass of a forward product from v also applies a pending f, w update (SC_UPD)
// to its output voxels (nx % 4 == 0). fin >= 0 (nx % 4 == 0): each instance also gets a
// finaliser block that runs finaliser fin (Fin) on its fin_n partials (per instance from fin_np
// when fin_np.n > 0) of an earlier launch; a uniform launch adds the block itself, a ragged map
// must count it (the last block of each instance's range).
int launch_blur_x(hipStream_t st, InstDesc *const *d, int B, long long n, int nx, int src, int dst,
                  int adj, int epi, int groups, const Rag &rg = kNoRag, int upd = 0, int fin = -1,
                  int fin_n = 0, const Rag &fin_np = kNoRag);
// y (axis 1) or z (axis 2) pass; window: outputs per thread along the axis (4, 8, 16 or 32;
// 0: default). upd: the pass applies a pending f, w update to its output voxels (the second pass
// of a forward product whose first pass carries a finaliser block).
int launch_blur_axis(hipStream_t st, InstDesc *const *d, int B, int nx, int ny, int nz, int axis,
                     int src, int dst, int adj, int epi, int window, const Rag &rg = kNoRag,
                     int upd = 0);
// blocks per instance of the passes above
int blur_x_blocks(long long n, int nx, int groups);
int blur_axis_blocks(int nx, int ny, int nz, int axis, int window);
int launch_gemv_rows(hipStream_t st, InstDesc *const *d, int B, long long m, int src, int epi,
                     int rows);
void launch_gemv_cols(hipStream_t st, InstDesc *const *d, int B, long long n, int chunks);
void launch_colsum(hipStream_t st, InstDesc *const *d, int B, long long n, int epi);
int launch_copy_g_u(hipStream_t st, InstDesc *const *d, int B, long long m);
// np: per-instance partial counts of a ragged producer (then one block per entry), or kNoRag
void launch_finalize(hipStream_t st, InstDesc *const *d, int B, int nparts, int what,
                     const Rag &np = kNoRag);
void launch_init_wf(hipStream_t st, InstDesc *const *d, int B, long long n);
// pending_only: only where the last MLSQR step left its update pending (SC_UPD)
void launch_update_fw(hipStream_t st, InstDesc *const *d, int B, long long n,
                      const Rag &rg = kNoRag, int pending_only = 0);
int launch_dot_vp(hipStream_t st, InstDesc *const *d, int B, long long n);
// batched dense products on MFMA (gemm_bf16.hip)
// upd: the packing also applies a pending f, w update (SC_UPD) of the product's instances
int launch_gemm_forward(hipStream_t st, InstDesc *const *d, int B, const GemmArgs &g, long long m,
                        long long n, int src_sel, int epi, int upd = 0);
void launch_gemm_adjoint(hipStream_t st, InstDesc *const *d, int B, const GemmArgs &g, long long m,
                         long long n, int epi);
// Tiled BF16 left operands of the batched products (n_y, n_x divisible by 256), stored as
// interleaved hi/lo tile pairs (2 x n_y x n_x bf16): the split hi = bf16(L), lo = bf16(L - hi)
// of L = A (transposed = 0) or L = A^T (transposed = 1) from the float32 row-major A, or the
// tiled copy of a 16-bit row-major A into the pairs' hi (part 0) or lo (part 1) halves.
void launch_split_tiled(hipStream_t st, const float *A, long long n_y, long long n_x,
                        int transposed, void *dst);
void launch_retile16(hipStream_t st, const void *src, long long n_y, long long n_x,
                     int transposed, int part, void *dst);
void launch_copy_out(hipStream_t st, InstDesc *const *d, int B, long long n);
// matrix-free ring sensitivity products (ring.hip); the forward returns its partial count
int launch_ring_forward(hipStream_t st, InstDesc *const *d, int B, const InstDesc &H, int src,
                        int epi);
void launch_ring_adjoint(hipStream_t st, InstDesc *const *d, int B, const InstDesc &H, int epi);
// several dampings from one Krylov run (kernels.hip)
void launch_basis_store(hipStream_t st, InstDesc *const *d, int B, long long n);
void launch_tau_finish(hipStream_t st, InstDesc *const *d, int B, long long n, int n_tau);
// S4 residual recurrence (kernels.hip)
void launch_s4_begin(hipStream_t st, InstDesc *const *d, int B, long long m);
int launch_s4_step(hipStream_t st, InstDesc *const *d, int B, long long m);

}  // namespace plsqr
