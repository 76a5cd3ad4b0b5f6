// solver.hpp -- batched solver internals shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "crdot.hpp"
#include "rbws_internal.hpp"

namespace rbws {

// one problem (grid) of a batch, as the kernels see it
struct ProbDev {
  GridDev g;
  int TX, TY, TZ, ntx, nty, ntz, ntiles, f_kind;
  double h, h2, gw;
};

// one solve of a batch
struct SolveDev {
  int prob, ntiles, item0, pad;
  long long off;      // offset of the solve's vectors, in elements
  long long kap_off;  // offset of its face-class coefficient table, in elements
  double x0[3];       // centre of the Gaussian source
};

// per-solve state of the FP32-inner / FP64-outer refinement (device memory)
struct IrState {
  double thr, ff, tol2, rr, init_rr, scale, upd, eta2;
  double rho, alpha, beta, thr_in, bb;
  int outer, mode, first, status, cur, k_in, k_total, restart, skip2, inner_max, max_outer, prec;
  unsigned long long t_done;
  double rescale;  // scale after / scale before the last outer correction (a power of two)
  int reliable;    // keep the search direction across outer corrections
  int dir_ok;      // the last inner solve ended with a usable direction
  int mg;          // the inner preconditioner is a V-cycle (s, r^T s follow the sweeps)
  int nvc;         // V-cycles applied
};

// partial results of a work item: FP64 path kSlots correctly rounded
// accumulators; refinement: IrPart (slot use documented at the kernels)
constexpr int kSlots = 3;
struct IrPart {
  CrAcc rr, ff;
  double g[3];
  double pad;
};

// device arrays of a batch (grow-only allocations, reused across calls)
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
  void* get(size_t need, int dev);
  void release();
  ~DevBuf() { release(); }
};

// function-local scratch that lives until the process ends (never freed, so no
// HIP call runs during static destruction)
#define RBWS_SCRATCH(name) static thread_local DevBuf& name = *new DevBuf()

void fill64(double* x, long long n, double v, hipStream_t s);

// Work lists of the iteration rounds.  Each round runs three sweeps: the A p
// sweep over the tiles of solves in CG iterations (ap), the residual sweep of
// solves whose residual is (re)evaluated (res), and the update sweep (up).  The
// per-solve finalisers append each unfinished solve's tiles to the list of the
// sweep it needs next, so a sweep touches active tiles only and the work of a
// shrinking batch stays spread over all XCDs.  cnt[WL_*] holds the lengths.
// The V-cycle of a multigrid-preconditioned solve runs over a list of the
// solves that need it this round, one segment per problem of the batch:
// mg[seg[q] ...] holds group-local indices (gidx[b] is solve b's index within
// its problem's group) and cnt[WL_MG + q] their number.
enum { WL_AP = 0, WL_RES = 1, WL_UP = 2, WL_MG = 8, WL_SEG = 32, WL_MAXPROB = 24 };
struct Lists {
  int* cnt;
  int* res;
  int* ap;
  int* up;
  int* mg;
  int* gidx;
};

struct Batch {
  int device = 0;
  int nsolve = 0, nprob = 0, nitems = 0;
  bool vec = true;      // every grid size is a multiple of 4 (vector loads)
  long long total = 0;      // sum of ndof over solves
  long long kap_total = 0;  // sum of table sizes
  int kap_max = 0;          // largest table (elements), for LDS sizing
  std::vector<const Problem*> probs;
  std::vector<ProbDev> pd_h;
  std::vector<SolveDev> sd_h;
  std::vector<int2> items_h;
  std::vector<double> theta_h;  // nsolve x kMaxQ
  DevBuf pd, sd, items, kap64, kap32, theta, ncorner, thidx, state, part, active, lists;
  std::vector<int> lists_h;  // initial list image: counts, then res = all items
  // FP64 CG vectors (sv: the preconditioned residual s when P is a V-cycle)
  DevBuf x, r, p, p2, sv, need;
  // FP32 inner vectors (refinement; sv32: s from the V-cycle)
  DevBuf d32, r32, p32, p32b, sv32;
  DevBuf fc;  // FP64 f_h of parameter-dependent sources (refinement outer passes)
  int* active_host = nullptr;  // pinned
  ~Batch();
};

// tiles: 256 threads of 4 x-points each, 32 x 32 grid columns, or a whole row
// (64 x 16, 128 x 8) when 32 < n <= 128, by TZ planes; TZ is the largest power
// of two in [4, 64] that still gives >= 4096 work items.  With `internal`
// (the coarser multigrid levels) the caller's fixed depth does not apply:
// those grids are too small for the depth chosen for the finest one.
void choose_tile(int n, long long nsolve_of_this_size, int* TX, int* TY, int* TZ, bool internal = false);
// autotuner of the tile depth (see solver.hip); its choices override the rule above
int autotune_tiles(const Problem* P, int nsolve, bool fp32, hipStream_t s, double* ms);
void clear_tile_table();
// fixed tile depth for every later batch (a power of two in [4, 64]), 0: automatic
void set_tile_depth(int tz);

// Lists with every item on the residual list and the others empty (stream-ordered)
Lists lists_init(Batch& B, hipStream_t s);

// Grid for a sweep kernel over up to `nitems` work items, a multiple of 8: one
// workgroup per item, or (grid_mode 1) as many 256-thread workgroups as fit on
// the device at once (occupancy with `lds` bytes of dynamic LDS), each looping
// over several items.
unsigned persistent_grid(const void* fn, size_t lds, int nitems, int device);
// 0: sweep grids have one workgroup per work item (the hardware dispatcher
// balances the load); 1: persistent grids.  RBWS_GRID overrides the default.
int grid_mode();
void set_grid_mode(int v);

// build the batch description: problems[prob_of[b]] for solve b; mu (nsolve x p) on host
// theta_override (nsolve x Q of problem 0, host) replaces theta(mu) when given;
// internal: tiles by choose_tile's own rule (coarser multigrid levels)
void batch_setup(Batch& B, const std::vector<const Problem*>& probs, const int* prob_of, int nsolve,
                 const double* mu, int p, hipStream_t s, const double* theta_override = nullptr,
                 bool internal = false);

// ||f - A x_b|| / ||f|| per solve for the x in `x` (laid out like the batch);
// rr and ff (correctly rounded) are returned too.  Host outputs.
void resid_norms(Batch& B, const double* x, double* rel, double* rr, double* ff, int force_exact,
                 hipStream_t s);

// FP64 PCG (Alg. 1) over all solves of the batch from the x already in B.x.
// Results: B.x (solutions), states in B.state.
struct CgOpts {
  double tol;
  int maxit, prec, flags, check_every;
  int mg_nu = 1;
  double mg_omega = 6.0 / 7.0;
};
void cg_fp64_run(Batch& B, const CgOpts& o, hipStream_t s);
void states_to_host(Batch& B, std::vector<CgState>& out, hipStream_t s);

// y = A x for every solve (FP64 or FP32), x/y laid out like the batch
void spmv_batch(Batch& B, const void* x, void* y, bool fp32, hipStream_t s);

// FP32-inner / FP64-outer refinement from the x already in B.x
struct IrOpts {
  double tol, eta;
  int prec, inner_max, max_outer, flags, check_every, reliable;
  int mg_nu = 1;
  double mg_omega = 6.0 / 7.0;
};
struct IrHost {
  int iters, outer, status, cur, nvc, pad;
  double init_rr, rr, ff;
  unsigned long long t_done;
};
// On return the solution of solve b is in (cur ? B.r : B.x) at its offset.
void ir_run(Batch& B, const IrOpts& o, hipStream_t s, std::vector<IrHost>& out);
int sweep32_variant();
void set_sweep32_variant(int v);

// The iteration rounds of a batched solve: `round(stream)` enqueues the launches
// of one round.  Rounds run until the device counter `active` reads 0 (checked
// every `check` rounds) or max_rounds.  With `graph`, `check` rounds are
// captured once into a HIP graph on a library stream (ordered after and before
// `s` by events) and the graph is replayed; otherwise the launches go to `s`.
// The rounds contain kernel launches only (no memset or copy nodes).
struct RoundStreams {
  hipStream_t ws = nullptr;
  hipEvent_t in = nullptr, out = nullptr;
};
RoundStreams& round_streams(int device);

template <class F>
void run_rounds(Batch& B, const int* active, long long max_rounds, int check, bool graph, hipStream_t s, F round) {
  if (!graph) {
    for (long long r = 0; r < max_rounds; r++) {
      round(s);
      RBWS_HIP(hipGetLastError());
      if ((r + 1) % check == 0) {
        RBWS_HIP(hipMemcpyAsync(B.active_host, active, sizeof(int), hipMemcpyDeviceToHost, s));
        RBWS_HIP(hipStreamSynchronize(s));
        if (*B.active_host == 0) break;
      }
    }
    return;
  }
  RoundStreams& rs = round_streams(B.device);
  RBWS_HIP(hipEventRecord(rs.in, s));
  RBWS_HIP(hipStreamWaitEvent(rs.ws, rs.in, 0));
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  RBWS_HIP(hipStreamBeginCapture(rs.ws, hipStreamCaptureModeThreadLocal));
  try {
    for (int r = 0; r < check; r++) round(rs.ws);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(rs.ws, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  RBWS_HIP(hipStreamEndCapture(rs.ws, &g));
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  const long long reps = (max_rounds + check - 1) / check;
  for (long long k = 0; k < reps && e == hipSuccess; k++) {
    e = hipGraphLaunch(ex, rs.ws);
    if (e == hipSuccess) e = hipMemcpyAsync(B.active_host, active, sizeof(int), hipMemcpyDeviceToHost, rs.ws);
    if (e == hipSuccess) e = hipStreamSynchronize(rs.ws);
    if (e == hipSuccess && *B.active_host == 0) break;
  }
  if (ex) (void)hipGraphExecDestroy(ex);
  (void)hipGraphDestroy(g);
  RBWS_HIP(e);
  RBWS_HIP(hipEventRecord(rs.out, rs.ws));
  RBWS_HIP(hipStreamWaitEvent(s, rs.out, 0));
}

// correctly rounded dots of `count` pairs of length len (device vectors)
void exact_dots(const double* x, const double* y, long long len, int count, double* out_host,
                int flags, hipStream_t s);
// the same into device memory, partial sums in a fixed static workspace:
// no allocation, no host synchronisation
void exact_dots_noalloc(const double* x, const double* y, long long len, int count, double* out_dev,
                        int flags, hipStream_t s);

// plain device copy (16-byte non-temporal loads and stores); bytes % 16 == 0
void stream_copy(const void* src, void* dst, long long bytes, hipStream_t s);

double wall_clock_khz(int device);

// Opt-in HIP-event timing of every launch of the solver's kernels, by kind.
enum KernelKind { KK_AP = 0, KK_RESID = 1, KK_FIN1 = 2, KK_UP2 = 3, KK_FIN2 = 4, KK_SPMV = 5, KK_LIFT = 6,
                  KK_COEF = 7, KK_MG = 8, KK_MG_PRE = 9, KK_MG_POST = 10, KK_PROJ = 11, KK_COUNT = 12 };
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> kind;  // per pair of events
  size_t used = 0;        // events in use
  double ms[KK_COUNT] = {};
  long long count[KK_COUNT] = {};
  void begin(hipStream_t s, int k);
  void end(hipStream_t s);
  void flush();           // wait for the recorded events and accumulate
};
KernelTimer& ktimer();

// exact-path fallback counters (diagnostics), per translation unit
unsigned long long fallbacks_solver(bool reset);
unsigned long long fallbacks_rb(int which, bool reset);

}  // namespace rbws
