/*
 * plsqr.h -- C ABI of the MI355X (gfx950) priorconditioned LSQR library.
 *
 * The library solves the edge-preserving regularised linear inverse problem
 *     min_f  1/2 ||g - A f||^2 + tau R(f),   R(f) = sum_j r(|grad f|_j)
 * (the MAP estimate of Section 1.1, eq. (1.6), with r from eq. (1.3)-(1.5)) by the
 * priorconditioned lagged-diffusivity method: Algorithm 3 (outer loop: freeze the
 * diffusivity kappa = r'(t)/t of eq. (1.12)-(1.13) at the previous iterate) around
 * Algorithm 2 (MLSQR, factorization-free priorconditioned LSQR) with the damping of
 * Section 3.3 / eq. (3.6), where the solve with the prior matrix
 *     M = G^T diag(kappa) G + eps I   (G: forward differences, zero at the upper
 *                                      boundary, i.e. the Neumann condition of (1.12))
 * is replaced by one geometric-multigrid V-cycle, a fixed SPD operator (Section 4.2).
 * Iteration counts are fixed (`outer` lagged-diffusivity steps x `inner` MLSQR steps)
 * unless the adaptive stops of the paper are requested (PLSQR_FLAG_STOP_S4,
 * PLSQR_FLAG_STOP_OUTER), which make the counts caps.
 *
 * Conventions
 *  - Grids are (nx, ny, nz), x fastest, float32, contiguous; nz == 1 is a 2D image.
 *  - Every call returns an int status (PLSQR_OK = 0, errors < 0); no exception crosses
 *    the ABI. plsqr_last_error() returns a message for the calling thread's last error.
 *  - Pointers named *_dev are device pointers on the engine's device; they are
 *    BORROWED: the caller keeps them alive (and, for inputs, unchanged) until the
 *    request that uses them has completed (plsqr_poll returned something other than
 *    PLSQR_PENDING), and for operators until plsqr_destroy.
 *  - Host pointers are read during the call only and may be freed afterwards.
 *  - An engine is driven by one host thread at a time (calls are serialised by an
 *    internal lock); work runs on the stream given at creation, in submission order.
 */
#ifndef PLSQR_H
#define PLSQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------- */
enum {
  PLSQR_OK = 0,
  PLSQR_PENDING = 1,            /* plsqr_poll: request not finished yet */
  PLSQR_E_INVALID = -1,         /* bad argument (sizes, enum values, null pointers) */
  PLSQR_E_NOMEM = -2,           /* device allocation failed */
  PLSQR_E_BUDGET = -3,          /* request can never fit the engine's HBM budget */
  PLSQR_E_HIP = -4,             /* a HIP runtime call failed */
  PLSQR_E_NOT_SPD = -5,         /* preconditioner or coarsest matrix not positive definite */
  PLSQR_E_NONFINITE = -6,       /* NaN/Inf met in the Krylov scalars (e.g. NaN in g) */
  PLSQR_E_UNKNOWN_TICKET = -7   /* ticket never issued, or already retired */
};

/* ---- enumerations ---------------------------------------------------------------- */
enum { PLSQR_OP_BLUR = 1, PLSQR_OP_DENSE = 2, PLSQR_OP_RING = 3 };
/* r(t) of eq. (1.3) (Tikhonov), (1.4) smoothed TV, (1.5) Perona-Malik log / exp forms */
enum { PLSQR_REG_TIKHONOV = 0, PLSQR_REG_STV = 1, PLSQR_REG_PM_LOG = 2, PLSQR_REG_PM_EXP = 3 };
enum { PLSQR_SMOOTH_JACOBI = 0, PLSQR_SMOOTH_CHEBYSHEV = 1 };
/* V-cycle launch schedule (plsqr_problem.tune_vcycle) */
enum { PLSQR_VCYCLE_FUSED = 0, PLSQR_VCYCLE_PER_SWEEP = 1 };
/* Where the f, w update of an MLSQR step runs on a blur operator (plsqr_problem.
 * tune_update_site; Algorithm 2's update, which nothing reads before the outer step ends):
 * AUTO picks the tail where it applies and the batch holds at most 2^22 voxels, else the
 * product; PRODUCT: in the next forward product's first or second pass; TAIL: in extra
 * workgroups of the next V-cycle's one-workgroup tail launch, which leaves most of the chip idle
 * (fused V-cycle, blur operator with nx % 4 == 0; elsewhere PRODUCT). The values are the same. */
enum { PLSQR_UPDATE_AUTO = 0, PLSQR_UPDATE_PRODUCT = 1, PLSQR_UPDATE_TAIL = 2 };
/* FP32: float32 vectors and products, float64 Krylov scalars and coarsest solve.
 * BF16_REFINED / BF16 (batches on a dense operator only): the dense products of the
 * batch run as BF16 MFMA GEMMs with FP32 accumulation. Every FP32 operand v is split
 * v = hi + lo (hi = bf16(v), lo = bf16(v - hi)); BF16_REFINED keeps the terms
 * A_hi X_hi + A_hi X_lo + A_lo X_hi (one refinement step of the BF16 product, error
 * ~2^-16 relative per entry), BF16 keeps A_hi X_hi + A_hi X_lo (A read once, error
 * ~2^-9 relative per entry of A). Vectors, stencils and scalars stay FP32/FP64. */
enum { PLSQR_PREC_FP32 = 0, PLSQR_PREC_BF16_REFINED = 1, PLSQR_PREC_BF16 = 2 };

/* engine creation flags */
enum {
  PLSQR_ENGINE_SERVE = 1u << 0  /* run a scheduler thread that admits requests by HBM
                                   budget and advances all resident requests together
                                   (continuous batching); default: each request is
                                   enqueued whole on submission */
};

/* problem flags */
enum {
  PLSQR_FLAG_TIME_PRODUCTS = 1u << 0, /* time every launch of the forward/adjoint product
                                         kernels with HIP events; totals in plsqr_result */
  PLSQR_FLAG_NO_GRAPHS = 1u << 1,     /* launch every kernel eagerly instead of replaying the
                                         inner iteration as a captured HIP graph */
  PLSQR_FLAG_STOP_S4 = 1u << 2,       /* inner stop by the discrepancy principle S4 of
                                         Section 3.4: MLSQR ends after the first step i with
                                         ||g - A f_i|| <= eta * delta; `inner` stays the cap
                                         on steps per outer iteration (Section 4.1) */
  PLSQR_FLAG_STOP_OUTER = 1u << 3,    /* outer stop of Algorithm 3 (step 5): after outer step
                                         k >= outer_min, stop when
                                         R(f^k) - R(f^{k-1}) >= -outer_rtol * R(f^{k-1}),
                                         i.e. R no longer falls by more than the fraction
                                         outer_rtol (Section 4.3 uses 0.15; Section 5.3 stops
                                         once R stops decreasing, outer_rtol = 0); the result
                                         is f^k, `outer` stays the cap */
  PLSQR_FLAG_TIME_PHASES = 1u << 4    /* time every phase of the method with HIP events on the
                                         engine stream (implies PLSQR_FLAG_TIME_PRODUCTS): setup
                                         (a1-a3), products, priorconditioner V-cycles, updates and
                                         per-outer diagnostics; totals in plsqr_result. The events
                                         add a few microseconds per phase. A serving engine
                                         records no phase times. */
};

#define PLSQR_MAX_LEVELS 12
#define PLSQR_MAX_OUTER 64
#define PLSQR_MAX_RADIUS 16
#define PLSQR_MAX_COARSE 512     /* largest coarsest-grid size solved by dense Cholesky */
#define PLSQR_STATIC_SCRATCH_BYTES (64u << 20)   /* device scratch of plsqr_solve_static */

typedef struct plsqr_engine plsqr_engine;   /* opaque; owns all internal device state */

/* Forward map A: R^{nx*ny*nz} -> R^{n_y} (the method only needs its action and that
 * of A^T; Section 1).
 *  PLSQR_OP_BLUR : separable correlation with taps[0..2*radius] (taps[radius] is the
 *                  centre) along every axis of extent > 1, zero outside the grid,
 *                  n_y = nx*ny*nz. The adjoint uses the reversed taps. taps is a HOST
 *                  pointer copied during the call. radius <= PLSQR_MAX_RADIUS.
 *  PLSQR_OP_DENSE: A_dev is a row-major n_y x (nx*ny*nz) float32 DEVICE matrix
 *                  (BORROWED). A_hi_dev / A_lo_dev are optional bf16 (uint16 bit
 *                  pattern) copies with the same layout: A_hi = bf16(A),
 *                  A_lo = bf16(A - A_hi). The batched BF16 products (PLSQR_PREC_BF16,
 *                  PLSQR_PREC_BF16_REFINED) take their operands from them when given
 *                  (else from A), copied once into library-owned tiled buffers when the
 *                  first such batch starts: hi and lo parts of A and of A^T, 4 x n_y x
 *                  nx*ny*nz x 2 bytes of device memory held until plsqr_destroy.
 *  PLSQR_OP_RING : the dense source-detector sensitivity of PLSQR_OP_DENSE's workloads,
 *                  never stored: entry (s * n_det + d, j) is
 *                      exp(-mu (r_sj + r_dj)) / (r_sj r_dj + 1),
 *                  r_sj, r_dj the distances from voxel centre j = (x, y, z) (integer
 *                  coordinates, x fastest) to source s and detector d. src_xyz (3 n_src
 *                  floats) and det_xyz (3 n_det) are HOST pointers copied during the call;
 *                  n_y = n_src * n_det (at most 16384), mu > 0. The products recompute the
 *                  entries (a stand-in for a forward map available only by its action,
 *                  Section 1, as the FEM solves of Section 5 are).
 */
typedef struct {
  int32_t kind;
  int32_t nx, ny, nz;
  int32_t radius;
  int32_t reserved0;
  const float *taps;
  int64_t n_y;
  const float *A_dev;
  const uint16_t *A_hi_dev;
  const uint16_t *A_lo_dev;
  /* PLSQR_OP_RING */
  int32_t n_src, n_det;
  const float *src_xyz;
  const float *det_xyz;
  double mu;
} plsqr_operator;

/* One reconstruction. Grid must equal the operator's grid.
 *  reg, T        : regulariser r(t) and its parameter T > 0 (ignored for Tikhonov)
 *  tau >= 0      : prior weight; MLSQR damping is sqrt(tau) (Section 3.3)
 *  eps > 0       : shift making M = G^T diag(kappa) G + eps I positive definite
 *  outer, inner  : iteration counts (caps under the stop flags), 1 <= outer <= PLSQR_MAX_OUTER,
 *                  inner >= 1
 *  mg_levels     : number of grids (0: halve while every coarsened axis is even and
 *                  > 4); each coarsening halves nx, ny and (3D) nz, which must be even;
 *                  the coarsest grid must have <= PLSQR_MAX_COARSE cells
 *  smoother      : PLSQR_SMOOTH_JACOBI (damped, weight omega in (0,1]) with nu_pre = nu_post
 *                  sweeps, or PLSQR_SMOOTH_CHEBYSHEV (degree cheb_degree in D^{-1}A on
 *                  [cheb_lo, cheb_hi], applied nu_pre = nu_post times); equal pre and
 *                  post smoothing keeps the V-cycle symmetric (Section 4.2)
 *  precision     : PLSQR_PREC_*
 *  flags         : PLSQR_FLAG_*
 *  eta, delta    : with PLSQR_FLAG_STOP_S4, the discrepancy level eta * delta of S4 (delta:
 *                  the noise norm ||g - A f_true||, eta > 0, typically slightly above 1);
 *                  the residual ||g - A f_i|| is tracked through the recurrences
 *                  A w_{i+1} = A v_{i+1} - (theta/rho) A w_i, A f_i = A f_{i-1} + (phi/rho) A w_i
 *                  on two extra n_y vectors, so no extra product with A is spent
 *  outer_rtol,
 *  outer_min     : with PLSQR_FLAG_STOP_OUTER, the tolerance and first outer step
 *                  (2 <= outer_min) of the outer stop; ignored otherwise
 */
typedef struct {
  int32_t nx, ny, nz;
  int32_t reg;
  double T, tau, eps;
  int32_t outer, inner;
  int32_t mg_levels;
  int32_t smoother;
  int32_t nu_pre, nu_post;
  double omega;
  int32_t cheb_degree;
  int32_t precision;
  double cheb_lo, cheb_hi;
  uint32_t flags;
  /* performance knobs (0 = library default); they never change the method, only tiling:
   *  tune_gemv_rows   rows of A per block of the dense forward product (1, 2, 4 or 8)
   *  tune_col_chunks  row chunks of the dense adjoint product (1..64)
   *  tune_blur_window outputs per thread of the y/z blur passes (4, 8, 16 or 32; default 8)
   *  tune_blur_xgroups 4-output groups per thread of the x blur pass (1, 2 or 4; default 2)
   *  tune_vcycle      PLSQR_VCYCLE_FUSED (default): every level above the one-workgroup tail
   *                   runs its pre-smoothing with the residual restriction as one launch and its
   *                   prolongation with the post-smoothing as another (Jacobi with nu <= 4,
   *                   Chebyshev with nu = 1 and degree <= 4, levels with nx % 4 == 0);
   *                   PLSQR_VCYCLE_PER_SWEEP: one launch per sweep and a separate restriction.
   *                   Both compute the same values.
   *  tune_zm_ty, tune_zm_zc  output rows and planes per block of the fused level kernels
   *                   (even, ty in [2, 64], zc in [2, 64]; 0: chosen from the grid)
   *  tune_zm_v        voxels per thread of the fused level kernels, 1 or 4 (0: 4 on levels of
   *                   at least 2^20 cells, 1 below)
   *  tune_tail_cells  largest level (in cells) that joins the one-workgroup V-cycle tail
   *                   (0: 4096; at most 2^20)
   *  tune_update_site where the f, w update runs: PLSQR_UPDATE_AUTO (0), _PRODUCT or _TAIL */
  int32_t tune_gemv_rows;
  int32_t tune_col_chunks;
  /* adaptive stopping (PLSQR_FLAG_STOP_S4, PLSQR_FLAG_STOP_OUTER) */
  double eta, delta;
  double outer_rtol;
  int32_t outer_min;
  int32_t tune_blur_window;
  int32_t tune_blur_xgroups;
  int32_t tune_vcycle;
  int32_t tune_zm_ty;
  int32_t tune_zm_zc;
  int32_t tune_zm_v;
  int32_t tune_tail_cells;
  int32_t tune_update_site;
} plsqr_problem;

/* Completion record of one request (filled by plsqr_poll). */
typedef struct {
  int32_t status;                     /* PLSQR_OK or the request's error code */
  int32_t outer_done;                 /* outer iterations run (< outer after an outer stop) */
  int32_t levels;                     /* multigrid levels used */
  int32_t mixed_steps;                /* serving mode: inner steps that ran in launches shared
                                         with requests of other grids */
  int32_t inner_done[PLSQR_MAX_OUTER];/* MLSQR steps completed per outer iteration
                                         (< inner after an S4 or exact-termination stop) */
  double resid[PLSQR_MAX_OUTER];      /* ||g - A f^k|| per outer iteration k */
  double penalty[PLSQR_MAX_OUTER];    /* R(f^k) per outer iteration k */
  double submit_to_done_ms;           /* host wall time from plsqr_solve to completion
                                         being observed */
  double device_ms;                   /* device time of the request (HIP events) */
  double forward_ms;                  /* with PLSQR_FLAG_TIME_PRODUCTS: summed device time of
                                         the forward-product launches (A x) ... */
  int64_t forward_launches;           /* ... and their count */
  double adjoint_ms;                  /* same for the adjoint products (A^T u) */
  int64_t adjoint_launches;
  int64_t workspace_bytes;            /* device memory the request held */
  /* with PLSQR_FLAG_TIME_PHASES: summed device time of each phase (events around each phase
     on the engine stream; the launch gaps between phases are not counted, so the phases and
     the two product totals above add up to at most device_ms):
       setup_ms   diffusivity and penalty of the previous iterate, multigrid hierarchy and
                  coarsest factor, MLSQR initialisation (eq. (1.12)-(1.13), Section 4.2,
                  Algorithm 2 initialisation), once per outer step
       vcycle_ms  the inner steps' priorconditioner solves v = B p (one V-cycle, Section 4.2)
                  with the reduction alpha = sqrt(v.p) and the damping and Givens rotations
       update_ms  the inner steps' updates of f and w (and the S4 residual recurrence); for a
                  blur operator with nx % 4 == 0 and the fused V-cycle, the next forward
                  product (its time is part of forward_ms) or the next V-cycle's tail launch
                  (part of vcycle_ms, tune_update_site) applies the update
       diag_ms    the per-outer residual ||g - A f^k|| and penalty R(f^k), and the final copy
       phase_launches  inner steps timed */
  double setup_ms;
  double vcycle_ms;
  double update_ms;
  double diag_ms;
  int64_t phase_launches;
} plsqr_result;

/* Create an engine on HIP device `device`, with at most `hbm_budget_bytes` of
 * internal device memory (0 = no limit) and work submitted to `hip_stream`
 * (a hipStream_t, or NULL for the null stream). flags: PLSQR_ENGINE_*.
 * On success *out receives the engine; on error *out is NULL. */
int plsqr_create(plsqr_engine **out, int device, uint64_t hbm_budget_bytes, void *hip_stream,
                 uint32_t flags);

/* Register a forward operator (see plsqr_operator); *op_id receives its handle. */
int plsqr_set_operator(plsqr_engine *eng, const plsqr_operator *op, int32_t *op_id);

/* Submit one reconstruction: g_dev (n_y floats) is the data, f_dev (nx*ny*nz floats)
 * receives f^outer. Validates, then returns at once with *ticket; the work runs
 * asynchronously. f_dev is written only if the request succeeds. A request larger
 * than the whole budget fails with PLSQR_E_BUDGET; one that does not fit the memory
 * left waits until earlier requests complete. */
int plsqr_solve(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob, const float *g_dev,
                float *f_dev, uint64_t *ticket);

/* Several dampings from one Krylov run (Section 3.3). Runs as plsqr_solve (f_dev receives
 * f^outer for prob->tau; outer steps 1..outer-1 use prob->tau), and in the last outer step
 * keeps the vectors of the bidiagonalisation, which does not depend on tau: for each
 * taus[t] (HOST array of n_tau values >= 0, copied during the call) the projected problem
 * (3.6) is solved and f(taus[t]) = V y written to row t of f_taus_dev (DEVICE, n_tau x n_X
 * floats, BORROWED like f_dev, written only on success). 1 <= n_tau <= 64, inner <= 1024,
 * no stop flags, not on a serving engine. The extra workspace is inner x n_X floats. */
int plsqr_solve_taus(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob,
                     const float *g_dev, float *f_dev, int32_t n_tau, const double *taus,
                     float *f_taus_dev, uint64_t *ticket);

/* Submit `count` reconstructions that run in lockstep on one operator (one set of
 * launches serves all of them; with a BF16 precision the dense products become MFMA
 * GEMMs over the batch, reading A once per product for the whole batch). The problems
 * may differ in reg, T, tau, eps, omega and the Chebyshev interval but must share grid,
 * counts, levels, smoother kind and steps, precision and flags. BF16 batches need a
 * dense operator, count <= 64 and n_X, n_Y divisible by 256; the library builds tiled
 * BF16 copies of A and A^T (hi and lo parts) on first use, from the operator's
 * A_hi_dev / A_lo_dev when given, else from A, and keeps them until plsqr_destroy
 * (4 x n_Y x n_X x 2 bytes of device memory). tickets[i] receives the
 * ticket of request i; every ticket completes when the whole batch does. */
int plsqr_solve_batch(plsqr_engine *eng, int32_t op_id, int32_t count, const plsqr_problem *probs,
                      const float *const *g_devs, float *const *f_devs, uint64_t *tickets);

/* For callers that cannot allocate memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. One reconstruction as plsqr_solve runs it
 * (FP32, fixed or adaptive counts), with every internal buffer of the request (descriptor,
 * FP64 scalars and per-outer records, Krylov vectors, multigrid levels, reduction partials)
 * taken from a static device array of PLSQR_STATIC_SCRATCH_BYTES (64 MiB) that the library
 * holds on each GPU until the process ends. The call makes no device or pinned allocation,
 * no event and no graph: its kernels are launched eagerly on the engine's stream, the
 * descriptor travels as a kernel argument, and the records are cleared by a kernel.
 *  - A problem whose workspace (plsqr_workspace_bytes) exceeds the array fails with
 *    PLSQR_E_BUDGET and nothing is enqueued; so do timing flags (PLSQR_FLAG_TIME_*), a
 *    precision other than PLSQR_PREC_FP32 (PLSQR_E_INVALID) and a serving engine.
 *  - out == NULL: returns PLSQR_OK once the work is enqueued (usable under stream capture);
 *    f_dev is written when the stream reaches the end, unless the request fails.
 *    out != NULL: waits for the engine's stream, fills *out (status, counts, per-outer
 *    ||g - A f^k|| and R(f^k), workspace_bytes; no timings) and returns the request's
 *    status.
 *  - Every call on a GPU shares that GPU's array, which keeps the last call's contents:
 *    calls that overlap on one GPU (other engines or streams, other host threads) race and
 *    corrupt each other; calls in one stream order are safe. Requests submitted through the
 *    other entry points use their own memory and do not touch the array.
 *  g_dev, f_dev are device pointers as for plsqr_solve. */
int plsqr_solve_static(plsqr_engine *eng, int32_t op_id, const plsqr_problem *prob,
                       const float *g_dev, float *f_dev, plsqr_result *out);

/* Non-blocking completion check: PLSQR_PENDING while the request runs; otherwise the
 * request's status (PLSQR_OK or an error), with *out filled (out may be NULL). A
 * ticket is retired after its first non-PENDING return. */
int plsqr_poll(plsqr_engine *eng, uint64_t ticket, plsqr_result *out);

/* Block until every submitted request has completed (results stay pollable). */
int plsqr_wait_all(plsqr_engine *eng);

/* Wait for in-flight work, free all internal state and the engine. NULL is a no-op. */
int plsqr_destroy(plsqr_engine *eng);

/* Message describing the calling thread's last error (never NULL). */
const char *plsqr_last_error(const plsqr_engine *eng);

/* Number of grids the automatic rule picks for (nx, ny, nz) (mg_levels = 0). */
int plsqr_auto_levels(int32_t nx, int32_t ny, int32_t nz);

/* Bytes of device workspace one request of this problem needs (for HBM budgeting);
 * 0 if the arguments are invalid (the problem is validated as plsqr_solve does, against an
 * operator of kind op_kind on the problem's grid). op_kind is PLSQR_OP_*, n_y the operator's
 * row count. */
uint64_t plsqr_workspace_bytes(const plsqr_problem *prob, int32_t op_kind, int64_t n_y);

#ifdef __cplusplus
}
#endif
#endif /* PLSQR_H */
