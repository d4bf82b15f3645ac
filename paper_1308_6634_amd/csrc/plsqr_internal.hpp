// Internal device-side layout shared by the HIP kernels and the host engine.
//
// One reconstruction ("instance") owns one contiguous workspace holding its Krylov
// vectors, its multigrid hierarchy, its FP64 scalar block and reduction partials. A
// POD descriptor (InstDesc) in that workspace records every pointer and parameter;
// kernels receive a device array of descriptor pointers and work on instance
// blockIdx.y, so one launch serves a whole batch of instances.
#pragma once
#include <cstdint>

#include "../../include/plsqr.h"

namespace plsqr {

constexpr int kMaxLevels = PLSQR_MAX_LEVELS;
constexpr int kMaxTaps = 2 * PLSQR_MAX_RADIUS + 1;
constexpr int kBlock = 256;          // threads per block for grid kernels (4 wave64)
constexpr double kTiny = 1e-300;     // exact-termination threshold for alpha, beta
constexpr int kRingMaxRows = 16384;  // n_src * n_det of a ring operator (u staged in LDS)
constexpr int kMaxTaus = 64;         // dampings of one multi-tau solve
constexpr int kMaxTauInner = 1024;   // MLSQR steps of a multi-tau solve (coefficients in LDS)

// FP64 scalar block of one instance (MLSQR state of Algorithm 2 with damping).
enum ScalarSlot : int {
  SC_ALPHA = 0,   // alpha_i (true value)
  SC_BETA,        // beta_i
  SC_RHOBAR,      // rho_bar_i
  SC_PHIBAR,      // phi_bar_i
  SC_SU,          // 1/beta_i: scale of the stored (unnormalised) u
  SC_SV,          // 1/alpha_i: scale of the stored p and v
  SC_CF,          // phi_i / rho_i   (f update)
  SC_CW,          // theta_{i+1} / rho_i (w update)
  SC_STOP,        // 1 once MLSQR ended in this outer step (breakdown or S4) or the outer
                  // loop has stopped
  SC_DONE,        // MLSQR steps completed in this outer step
  SC_STATUS,      // 0 or a PLSQR_E_* code (sticky for the whole request)
  SC_OUTER,       // current outer index k (0 before the first)
  SC_LAMBDA,      // sqrt(tau)
  SC_HALT,        // 1 once the outer stop has fired: later outer steps change nothing
  SC_S4R,         // ||g - A f_i|| of the last completed step (S4 recurrence)
  SC_UPD,         // 1 while the f, w update of the last completed step is pending: the next
                  // forward product applies it, or the tail of the next V-cycle (see
                  // fused_update and tail_update in the driver)
  SC_FINA,        // 1 while the alpha finaliser of the last V-cycle is pending: the partials of
                  // v.p wait in `part` for the next forward product's finaliser block (see
                  // fin_blocks in the driver)
  SC_COUNT = 17
};

// Per-outer diagnostic record layout (doubles).
enum DiagSlot : int { DG_RESID = 0, DG_PENALTY, DG_INNER, DG_STATUS, DG_COUNT = 4 };

struct LevelDesc {
  int nx, ny, nz, pad;
  long long n;
  float *x, *b, *r, *t, *s;          // iterate, rhs, residual and two scratch vectors
  float *wx, *wy, *wz;               // face weights to the +x/+y/+z neighbour (levels >= 1)
  float *dinv;                       // 1 / diag(A_l)
  double eps;                        // eps_l = 2^{d l} eps
};

// Tile of a level's fused kernels: tx x-columns, ty rows, zc planes per block, v voxels per
// thread; tx = 0: the level runs the per-sweep kernels.
struct ZmPlan {
  int tx, ty, zc, v;
};

struct InstDesc {
  int nx, ny, nz, levels;
  long long n;                       // n_X
  long long m;                       // n_Y
  int reg, op_kind, radius, smoother;
  int nu_pre, nu_post, cheb_degree, dims;
  float T, omega;
  double tau, eps;
  double cheb_theta, cheb_delta, cheb_sigma;
  float taps[kMaxTaps];
  float taps_rev[kMaxTaps];          // taps reversed (the adjoint's correlation weights)
  const float *g;                    // data (n_Y)
  const float *A;                    // dense operator (row-major n_Y x n_X) or null
  float *f, *u, *p, *v, *w, *kappa;  // Krylov vectors (u has n_Y entries)
  float *tmp1, *tmp2;                // blur pass buffers
  float *colpart;                    // dense adjoint: per-row-chunk column partial sums
  float *out_f;                      // caller's output
  double *sc;                        // scalar block (SC_COUNT)
  double *part;                      // per-block reduction partials
  double *cfac;                      // coarsest level: Cholesky factor, L^{-1}, A^{-1} (3 x nc x nc)
  double *diag;                      // (outer + 1) x DG_COUNT records
  int nc, colchunks;
  int gemv_rows;                     // rows of A per block of the dense forward product
  int blur_window;                   // outputs per thread of the y/z blur passes (0: default)
  int blur_xgroups;                  // 4-output groups per thread of the x pass (0: default)
  int vcycle_mode;                   // PLSQR_VCYCLE_FUSED or PLSQR_VCYCLE_PER_SWEEP
  int zm_ty, zm_zc, zm_v;            // fused level kernels: rows / planes per block, voxels per
                                     // thread (0: chosen per level)
  int tail_cells;                    // largest level of the one-workgroup tail (0: default)
  int update_site;                   // where a pending f, w update runs (PLSQR_UPDATE_*)
  int stop_flags;                    // PLSQR_FLAG_STOP_S4 | PLSQR_FLAG_STOP_OUTER bits
  int outer_min;                     // first outer step checked by the outer stop
  double s4_level;                   // eta * delta
  double outer_rtol;
  float *aw, *af;                    // S4 residual recurrence (n_Y each): see k_s4_step
  const float *ring;                 // ring sensitivity: 3 n_src source, 3 n_det detector coords
  float *ringpart;                   // ring forward product partials (ring_chunks x n_Y)
  float *ringpart2;                  // their sums over groups of chunks (ring_groups x n_Y)
  int n_src, n_det, ring_chunk, ring_chunks, ring_groups;
  float ring_mu;
  // several dampings from the last outer step's Krylov run (Section 3.3); n_tau = 0: off
  int n_tau, outer_count, inner_count;
  float *basis;                      // inner x n_X: the vectors v_1.. that f combines
  double *hist;                      // 2 x (inner + 1): alpha_1.., beta_1..
  double *tau_scr;                   // n_tau x inner x 3: rho, theta, phi / solution y
  float *ycoef;                      // n_tau x inner: f(tau_t) = sum_i ycoef[t][i] v_i
  float *f_taus;                     // caller's n_tau x n_X output
  double taus[kMaxTaus];
  // the fused V-cycle as the driver runs it (what a launch serving instances of different
  // grids reads per instance): each level's fused-kernel tile and the first level of the
  // LDS-resident tail
  ZmPlan zmp[kMaxLevels];
  int tail_lds_t;
  LevelDesc lv[kMaxLevels];
};

// Map of a ragged launch: blocks [first[k], first[k] + count[k]) of a one-dimensional grid
// serve instance inst[k] (an index into the launch's descriptor array); first[k] is a multiple
// of 8, and blocks outside every range return at once. n = 0: a uniform launch, where blockIdx.y
// is the instance and blockIdx.x the block within it. For k_finalize, count[k] is instance
// inst[k]'s partial count.
constexpr int kMaxRag = 32;
struct Rag {
  int n;
  int inst[kMaxRag], first[kMaxRag], count[kMaxRag];
};
inline constexpr Rag kNoRag{};

// Selectors for vectors inside an instance (kernels are batched, so they cannot take
// per-instance pointers directly).
enum VecSel : int { V_F = 0, V_U, V_P, V_V, V_W, V_TMP1, V_TMP2, V_G };

// Epilogues of the last pass of a forward/adjoint product.
enum Epi : int {
  EPI_STORE = 0,    // out = y
  EPI_FWD,          // u <- sv * y - (alpha * su) * u, partial ||u||^2
  EPI_ADJ,          // p <- su * y - (beta * sv) * p
  EPI_ADJ_INIT,     // p <- su * y
  EPI_RESID         // partial ||g - y||^2 (nothing stored)
};

// Mask bits or-ed into a product's epilogue code by the driver for problems with adaptive
// stops: the launch does nothing for an instance whose MLSQR has ended in this outer step
// (inner products) or whose outer loop has ended (the per-outer residual product).
constexpr int EPI_MASK_INNER = 0x100;
constexpr int EPI_MASK_OUTER = 0x200;

// Reduction finalisers (one block per instance). FIN_BETA_PEND: FIN_BETA, then marks the alpha
// finaliser of the V-cycle that follows as pending (SC_FINA); FIN_ALPHA_PEND: FIN_ALPHA if it is
// pending (and clears the mark), else nothing. The _T forms are for steps whose pending update
// runs in the V-cycle tail (after the beta finaliser): FIN_BETA_PEND_T leaves the update pending
// and FIN_ALPHA_PEND_T first retires it (that tail has run by then).
enum Fin : int {
  FIN_BETA_INIT = 0, FIN_BETA, FIN_ALPHA_INIT, FIN_ALPHA, FIN_RESID, FIN_PENALTY, FIN_S4,
  FIN_BETA_PEND, FIN_ALPHA_PEND, FIN_BETA_PEND_T, FIN_ALPHA_PEND_T
};

}  // namespace plsqr

namespace plsqr {
// Dense products of a lockstep batch on MFMA (BF16 operands, FP32 accumulation).
struct GemmArgs {
  const void *A_t;             // A (n_Y x n_X) as tiled bf16 hi/lo tile pairs (forward)
  const void *At_t;            // A^T (n_X x n_Y), the same layout (adjoint)
  void *X_hi, *X_lo;           // packed right operand, Bpad x n_X (forward)
  void *U_hi, *U_lo;           // packed right operand, Bpad x n_Y (adjoint)
  float *Ypart;                // forward split-K partials, ks x n_Y x Bpad
  int Bpad, ks;                // padded batch (multiple of 32), K splits of the forward GEMM
  long long kchunk;            // forward K chunk (multiple of 256)
  int use_A_lo;                // add the A_lo x X_hi refinement term
};
}  // namespace plsqr
