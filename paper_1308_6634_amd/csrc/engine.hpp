// Host engine: operators, requests, device workspaces and the solve driver.
#pragma once
#include <hip/hip_runtime_api.h>

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "plsqr_internal.hpp"

namespace plsqr {

struct Operator {
  plsqr_operator op{};
  std::vector<float> taps;
  // tiled BF16 left operands of the batched MFMA products, A and A^T, each holding its hi and
  // lo parts as interleaved tile pairs (built on first use, owned)
  void *A_t = nullptr, *At_t = nullptr;
  // ring sensitivity: source then detector positions (x, y, z floats) on the device
  float *ring = nullptr;
};

// Byte offsets of every buffer inside one request's workspace.
struct Layout {
  size_t total = 0;
  size_t desc = 0, descptr = 0, sc = 0, diag = 0, part = 0, cfac = 0;
  size_t f = 0, p = 0, v = 0, w = 0, kappa = 0, u = 0, tmp1 = 0, tmp2 = 0, colpart = 0;
  size_t aw = 0, af = 0;              // S4 residual recurrence vectors (n_Y), 0 when unused
  size_t ringpart = 0, ringpart2 = 0;  // ring forward product: per-chunk and per-group partials
  int ring_chunk = 0, ring_chunks = 0, ring_groups = 0;  // voxels per block, chunks, groups
  size_t basis = 0, hist = 0, tau_scr = 0, ycoef = 0;  // multi-tau solve, 0 when unused
  size_t lvl[kMaxLevels][10] = {};   // x b r t s wx wy wz dinv (unused slots 0)
  int nparts = 0, colchunks = 0, levels = 0, nc = 0;
  long long n = 0, m = 0;
  long long ln[kMaxLevels] = {};
  int lnx[kMaxLevels] = {}, lny[kMaxLevels] = {}, lnz[kMaxLevels] = {};
};

// Validate a problem against an operator; fills *levels. Returns PLSQR_OK or an error
// with a message in *why.
int validate(const plsqr_problem &pb, const Operator *op, int *levels, std::string *why);
Layout make_layout(const plsqr_problem &pb, long long n_y, int levels, int op_kind, int n_tau = 0);

// Workspace cache: freed workspaces are kept for reuse by requests of the same size.
class Pool {
 public:
  ~Pool();
  void *get(size_t bytes);
  void put(void *p, size_t bytes);
  void trim();
 private:
  std::multimap<size_t, void *> free_;
};

using EventList = std::vector<std::pair<hipEvent_t, hipEvent_t>>;

// Replayable HIP graphs of the inner iteration (plain and lockstep groups): captured once on
// a private stream, launched on the engine stream for every inner step.
struct GraphCache {
  hipStream_t cap = nullptr;                 // capture stream (non-blocking, default priority)
  std::vector<hipGraphExec_t> execs;
  ~GraphCache();
};
// One reconstruction.
struct Request {
  uint64_t ticket = 0;
  uint64_t group = 0;
  plsqr_problem pb{};
  const float *g = nullptr;
  float *f_out = nullptr;
  std::vector<double> taus;          // multi-tau solve: dampings and the caller's outputs
  float *f_taus = nullptr;
  Layout lay;
  char *ws = nullptr;                // device workspace
  InstDesc host{};                   // host copy of the descriptor
  InstDesc *d_desc = nullptr;        // device copy (in ws)
  char *pinned = nullptr;            // pinned staging: descriptor up, scalars/records down
  bool done = false;
  int status = PLSQR_OK;
  std::string err;   // why the request failed (set with a failing status)
  double t_submit = 0.0, t_done = 0.0;
  plsqr_result result{};
  // serving mode: position in the fixed step schedule and completion event
  int step = 0, steps_total = 0;
  int mixed_steps = 0;       // serving: inner steps run in launches shared with other grids
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
};

// Step types of the served schedule: BEGIN, then per outer iteration OUTER_START
// (setup + MLSQR initialisation), `inner` x INNER, OUTER_END, and finally FINISH.
enum StepType : int { ST_BEGIN = 0, ST_OUTER_START, ST_INNER, ST_OUTER_END, ST_FINISH };
inline int step_count(const plsqr_problem &pb) { return 2 + pb.outer * (pb.inner + 2); }
inline int step_type(const plsqr_problem &pb, int s) {
  if (s == 0) return ST_BEGIN;
  if (s == step_count(pb) - 1) return ST_FINISH;
  const int q = (s - 1) % (pb.inner + 2);
  return q == 0 ? ST_OUTER_START : (q <= pb.inner ? ST_INNER : ST_OUTER_END);
}

// Instances launched together in lockstep (a plain solve is a group of one).
struct Group {
  uint64_t id = 0;
  int op_id = 0;
  std::vector<uint64_t> members;
  int precision = PLSQR_PREC_FP32;
  enum State { QUEUED, RUNNING, DONE } state = QUEUED;
  size_t bytes = 0;                  // members' workspaces + group workspace
  char *gws = nullptr;               // group workspace: descriptor pointer array, MFMA buffers
  size_t gws_bytes = 0;
  InstDesc **d_descs = nullptr;
  char *pinned = nullptr;            // staging of the pointer array
  GemmArgs gemm{};
  bool use_gemm = false;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  EventList fwd_events, adj_events;
  // phase timing (PLSQR_FLAG_TIME_PHASES): setup, V-cycle, update and diagnostics phases
  EventList setup_events, vcycle_events, update_events, diag_events;
  bool timed = false;
  bool phases = false;
  std::unique_ptr<GraphCache> graphs;      // captured inner iteration (null: eager launches)
};

// A view of B same-shaped instances launched together.
struct BatchView {
  InstDesc *const *d_descs;   // device array of B descriptor pointers
  int B;
  const InstDesc *h;          // host copy of one member (shapes and schedule)
  const Layout *lay;
  EventList *prod_events;     // optional timing (forward products)
  EventList *adj_events;      // optional timing (adjoint products)
  const GemmArgs *gemm;       // batched MFMA products, or null
  // optional phase timing: events around the setup (a1-a3), inner V-cycle (with the alpha
  // reduction and rotations), inner update and per-outer diagnostics phases
  EventList *setup_events = nullptr;
  EventList *vcycle_events = nullptr;
  EventList *update_events = nullptr;
  EventList *diag_events = nullptr;
};

// Instances of different grids advanced by one inner step in shared launches (serving mode).
struct RagBatch {
  InstDesc *const *d_descs;   // device array of B descriptor pointers
  int B;                      // at most kMaxRag
  const InstDesc *const *h;   // host copy of each instance
  const Layout *const *lay;   // and its layout
};
// Whether an instance's inner step can share launches with instances of other grids: a 3D blur
// operator with nx % 4 == 0, the fused V-cycle on every level above its tail, no S4 stop and a
// single damping. Instances that share launches must also agree on the smoother schedule, the
// blur launch knobs and the stop flags.
bool ragged_ok(const InstDesc &H, const Layout &Ly);
void enqueue_inner_ragged(hipStream_t st, const RagBatch &rb);
// The fused V-cycle schedule of an instance (per-level fused tiles, first tail level) into its
// descriptor: what enqueue_vcycle runs for it.
void plan_vcycle(InstDesc &D, const Layout &Ly);

// Solve driver (same sequence for one instance or a lockstep batch).
void enqueue_request_begin(hipStream_t st, const BatchView &bv);
void enqueue_outer_setup(hipStream_t st, const BatchView &bv);
void enqueue_mlsqr_init(hipStream_t st, const BatchView &bv);
void enqueue_inner(hipStream_t st, const BatchView &bv);
void enqueue_outer_end(hipStream_t st, const BatchView &bv);
void enqueue_request_end(hipStream_t st, const BatchView &bv);
void enqueue_whole_solve(hipStream_t st, const BatchView &bv, int outer, int inner,
                         GraphCache *graphs);

double now_ms();

// Static scratch of the no-allocation entry point (static_scratch.hip): resolve_scratch looks
// up the array's device address on `device` (which must be current) once per device;
// scratch_ptr returns it (null before). launch_static_setup writes a request's descriptor and
// pointer array into it and clears the per-outer records.
int resolve_scratch(int device, std::string *why);
void *scratch_ptr(int device);
void launch_static_setup(hipStream_t st, const InstDesc &desc, InstDesc *d_desc, InstDesc **d_ptrs,
                         double *records, int n_records);

}  // namespace plsqr

struct plsqr_engine {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;      // 0 = unlimited
  uint64_t used = 0;
  uint32_t flags = 0;
  std::mutex mu;
  std::vector<plsqr::Operator> ops;
  std::map<uint64_t, std::unique_ptr<plsqr::Request>> reqs;
  std::map<uint64_t, std::unique_ptr<plsqr::Group>> groups;
  std::deque<uint64_t> queued;       // group ids in FIFO order
  uint64_t next_ticket = 1;
  uint64_t next_group = 1;
  plsqr::Pool pool;
  // serving mode (PLSQR_ENGINE_SERVE): scheduler thread state, all guarded by mu
  std::thread worker;
  std::condition_variable cv;
  bool stop_worker = false;
  std::deque<uint64_t> serve_queue;   // submitted, waiting for memory
  std::vector<uint64_t> resident;     // admitted, advancing one step per tick
  std::vector<uint64_t> finishing;    // last step enqueued, waiting for the device
  struct TickSlot {
    hipEvent_t ev = nullptr;
    char *pinned = nullptr;           // pointer arrays of the tick's subgroups (host)
    char *dev = nullptr;              // ... and their device copy
    size_t cap = 0;
  };
  std::vector<TickSlot> ring;
  std::deque<int> inflight;           // ring slots whose ticks are on the device
  std::vector<hipStream_t> lanes;     // worker streams: a tick's subgroups run concurrently
  std::vector<hipEvent_t> lane_done;  // per-lane end-of-tick events (joined on `stream`)
  hipEvent_t ev_upload = nullptr;     // pointer arrays of the tick are on the device
  int ring_next = 0;
  uint64_t ticks = 0;
  int max_inflight_ticks = 2;         // below the ring size (4): a reused slot has finished
};
