// solver.hip -- batched FP64 PCG on gfx950 (the paper's Alg. 1, P in {I, Jacobi}).
//
// One "round" advances every unfinished solve of the batch by one CG
// iteration, in five launches:
//   ap   : p = s + beta p (s = P(r); p = s after a (re)start) fused with
//          gamma = p^T A p, over the tiles of ITER solves
//   res  : r = f - A x, ||r||^2, r^T s, ||f||^2, over the tiles of RESID solves
//   fin1 : per solve: alpha = rho / gamma, or the convergence decision of a
//          residual evaluation (initial residual or true-residual confirmation)
//   up2  : x += alpha p, r -= alpha A p (A p recomputed), ||r||^2, r^T s
//   fin2 : per solve: convergence test on the recursive residual, beta
// The sweeps run a persistent grid over work lists that the finalisers fill
// (solver.hpp, Lists).  The matrix is never stored: face coefficients come
// from a per-solve class table in LDS (see problem.cpp), so a stencil
// application reads one vector.  Every inner product is correctly rounded
// (crdot.hpp); together with the fixed evaluation order of the stencil and of
// every vector update this makes each solve's trajectory independent of
// tiling, scheduling and batch composition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fast.hpp"
#include "mg.hpp"

namespace rbws {

enum { OP_AP = 1, OP_RNORM = 3 };
enum { DOT_PAP = 0, DOT_RR = 1, DOT_RS = 2, DOT_FF = 3, DOT_RESID = 4, DOT_RSV = 5 };

// exact-path fallbacks taken by this translation unit's kernels (diagnostics)
__device__ unsigned long long g_fallback_solver;

void* DevBuf::get(size_t need, int dev) {
  if (need == 0) need = 1;
  if (ptr && bytes >= need && device == dev) return ptr;
  release();
  RBWS_HIP(hipSetDevice(dev));
  hipError_t e = hipMalloc(&ptr, need);
  if (e != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    throw Error{RBWS_ENOMEM, "device allocation of " + std::to_string(need) + " bytes failed"};
  }
  bytes = need;
  device = dev;
  return ptr;
}

void DevBuf::release() {
  if (ptr) {
    (void)hipSetDevice(device);
    (void)hipFree(ptr);
  }
  ptr = nullptr;
  bytes = 0;
}

Batch::~Batch() {
  if (active_host) (void)hipHostFree(active_host);
}

RoundStreams& round_streams(int device) {
  static thread_local std::vector<RoundStreams*> per;  // never destroyed (no HIP calls at exit)
  if ((int)per.size() <= device) per.resize(device + 1, nullptr);
  if (!per[device]) {
    RoundStreams* r = new RoundStreams();
    RBWS_HIP(hipStreamCreateWithFlags(&r->ws, hipStreamNonBlocking));
    RBWS_HIP(hipEventCreateWithFlags(&r->in, hipEventDisableTiming));
    RBWS_HIP(hipEventCreateWithFlags(&r->out, hipEventDisableTiming));
    per[device] = r;
  }
  return *per[device];
}

Lists lists_init(Batch& B, hipStream_t s) {
  const int ni = B.nitems, ns = B.nsolve;
  const size_t head = 64;  // counters and segment offsets, padded
  int* base = (int*)B.lists.get(sizeof(int) * (head + 3 * (size_t)ni + 2 * (size_t)ns), B.device);
  // host image: head, res = all items, then (after ap and up, not copied) mg and gidx
  B.lists_h.assign(head + ni, 0);
  B.lists_h[WL_RES] = ni;
  for (int t = 0; t < ni; t++) B.lists_h[head + t] = t;
  std::vector<int> gidx(ns), seg(B.nprob + 1, 0);
  for (int b = 0; b < ns; b++) gidx[b] = seg[B.sd_h[b].prob + 1]++;
  for (int q = 0; q < B.nprob; q++) seg[q + 1] += seg[q];
  for (int q = 0; q < B.nprob && q < WL_MAXPROB; q++) B.lists_h[WL_SEG + q] = seg[q];
  B.lists_h.insert(B.lists_h.end(), gidx.begin(), gidx.end());  // kept: the copies are asynchronous
  int* mg = base + head + 3 * (size_t)ni;
  RBWS_HIP(hipMemcpyAsync(base, B.lists_h.data(), sizeof(int) * (head + ni), hipMemcpyHostToDevice, s));
  RBWS_HIP(hipMemcpyAsync(mg + ns, B.lists_h.data() + head + ni, sizeof(int) * ns, hipMemcpyHostToDevice, s));
  return Lists{base, base + head, base + head + ni, base + head + 2 * (size_t)ni, mg, mg + ns};
}

static int g_grid_mode = -1;
int grid_mode() {
  if (g_grid_mode < 0) {
    const char* e = std::getenv("RBWS_GRID");
    g_grid_mode = e ? (std::atoi(e) & 1) : 0;
  }
  return g_grid_mode;
}
void set_grid_mode(int v) { g_grid_mode = v & 1; }

unsigned persistent_grid(const void* fn, size_t lds, int nitems, int device) {
  const unsigned need = 8u * (unsigned)((std::max(nitems, 1) + 7) / 8);
  if (grid_mode() == 0) return need;
  struct Key {
    const void* fn;
    size_t lds;
    int dev;
  };
  struct Ent {
    Key k;
    unsigned blocks;
  };
  static thread_local std::vector<Ent> cache;
  unsigned cap = 0;
  for (const Ent& e : cache)
    if (e.k.fn == fn && e.k.lds == lds && e.k.dev == device) cap = e.blocks;
  if (cap == 0) {
    int per_cu = 0, cus = 0;
    RBWS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds));
    RBWS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    cap = (unsigned)std::max(1, per_cu) * (unsigned)std::max(1, cus);
    cap = std::max(8u, cap & ~7u);
    cache.push_back(Ent{Key{fn, lds, device}, cap});
  }
  return std::min(cap, need);
}

// tile depths found by the autotuner, per (grid size, log2 of the number of solves of that size)
struct TileEntry {
  int n, bucket, tz;
};
static std::vector<TileEntry> g_tiles;
static int g_force_tz = 0;  // set by the autotuner while it times a candidate
static int g_user_tz = 0;   // set by the caller (RBWS_TUNE_TZ); 0: automatic
void set_tile_depth(int tz) { g_user_tz = tz; }
static int count_bucket(long long c) {
  int b = 0;
  while ((2LL << b) <= std::max(1LL, c)) b++;
  return b;
}

void choose_tile(int n, long long nsolve_of_this_size, int* TX, int* TY, int* TZ, bool internal) {
  // one tile spans the whole row when 32 < n <= 128 (no x-halo, contiguous y-halo rows)
  *TX = n > 128 || n <= 32 ? QX : (n > 64 ? 128 : 64);
  *TY = 1024 / *TX;
  if (!internal && (g_force_tz > 0 || g_user_tz > 0)) {
    *TZ = std::min(g_force_tz > 0 ? g_force_tz : g_user_tz, n);
    return;
  }
  const int bk = count_bucket(nsolve_of_this_size);
  for (const TileEntry& e : g_tiles)
    if (e.n == n && e.bucket == bk) {
      *TZ = std::min(e.tz, n);
      return;
    }
  const long long cols = (long long)((n + *TX - 1) / *TX) * ((n + *TY - 1) / *TY) * std::max(1LL, nsolve_of_this_size);
  int tz = 64;
  while (tz > 4 && cols * ((n + tz - 1) / tz) < 4096) tz /= 2;
  *TZ = std::min(tz, n);
}

// Times the stencil sweep (y = A x over `nsolve` solves of problem P, in FP32
// or FP64) for every tile depth TZ in {4, 8, 16, 32, 64} (TZ <= n), keeps the
// fastest for batches with this grid size and a solve count in the same
// power-of-two range, and returns it.  ms[5] receives the mean time per
// launch of each depth's faster pass (0 for a depth that was not tried).
int autotune_tiles(const Problem* P, int nsolve, bool fp32, hipStream_t s, double* ms) {
  RBWS_REQUIRE(nsolve >= 1, RBWS_EINVAL, "nsolve < 1");
  RBWS_HIP(hipSetDevice(P->device));
  Batch B;
  std::vector<double> mu((size_t)nsolve * P->p, 1.0);
  if (P->desc.f_kind == RBWS_F_GAUSS)
    for (int b = 0; b < nsolve; b++)
      for (int t = P->p - 3; t < P->p; t++) mu[(size_t)b * P->p + t] = 0.5;
  std::vector<const Problem*> probs{P};
  const size_t el = fp32 ? sizeof(float) : sizeof(double);
  const long long tot = (long long)nsolve * P->ndof;
  DevBuf xb, yb;
  void* x = xb.get(el * tot, P->device);
  void* y = yb.get(el * tot, P->device);
  RBWS_HIP(hipMemsetAsync(x, 0, el * tot, s));
  hipEvent_t e0, e1;
  RBWS_HIP(hipEventCreate(&e0));
  RBWS_HIP(hipEventCreate(&e1));
  const int cand[5] = {4, 8, 16, 32, 64};
  int best = 0;
  double best_ms = 0.0;
  double tmin[5] = {0, 0, 0, 0, 0};
  try {
    // two interleaved passes over the depths, five launches each; a depth's
    // time is its faster pass (a single short pass can rank two depths within
    // a few per cent of each other either way)
    for (int pass = 0; pass < 2; pass++) {
      for (int c = 0; c < 5; c++) {
        if (cand[c] > P->n && c > 0 && cand[c - 1] >= P->n) continue;
        g_force_tz = cand[c];
        batch_setup(B, probs, nullptr, nsolve, mu.data(), P->p, s);
        g_force_tz = 0;
        spmv_batch(B, x, y, fp32, s);
        RBWS_HIP(hipEventRecord(e0, s));
        const int reps = 5;
        for (int r = 0; r < reps; r++) spmv_batch(B, x, y, fp32, s);
        RBWS_HIP(hipEventRecord(e1, s));
        RBWS_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        RBWS_HIP(hipEventElapsedTime(&t, e0, e1));
        const double m = t / reps;
        if (pass == 0 || m < tmin[c]) tmin[c] = m;
      }
    }
    for (int c = 0; c < 5; c++) {
      if (ms) ms[c] = tmin[c];
      if (tmin[c] > 0.0 && (best == 0 || tmin[c] < best_ms)) {
        best = cand[c];
        best_ms = tmin[c];
      }
    }
  } catch (...) {
    g_force_tz = 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int bk = count_bucket(nsolve);
  bool found = false;
  for (TileEntry& e : g_tiles)
    if (e.n == P->n && e.bucket == bk) {
      e.tz = best;
      found = true;
    }
  if (!found) g_tiles.push_back(TileEntry{P->n, bk, best});
  return best;
}

void clear_tile_table() { g_tiles.clear(); }

unsigned long long fallbacks_solver(bool reset) {
  unsigned long long v = 0;
  RBWS_HIP(hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_fallback_solver), sizeof v));
  if (reset) {
    const unsigned long long z = 0;
    RBWS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_fallback_solver), &z, sizeof z));
  }
  return v;
}

KernelTimer& ktimer() {
  static thread_local KernelTimer& t = *new KernelTimer();
  return t;
}

void KernelTimer::begin(hipStream_t s, int k) {
  if (!on) return;
  while (pool.size() < used + 2) {
    hipEvent_t e;
    RBWS_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  kind.push_back(k);
  RBWS_HIP(hipEventRecord(pool[used++], s));
}

void KernelTimer::end(hipStream_t s) {
  if (!on) return;
  RBWS_HIP(hipEventRecord(pool[used++], s));
  if (used >= 4096) flush();
}

void KernelTimer::flush() {
  if (used == 0) return;
  RBWS_HIP(hipEventSynchronize(pool[used - 1]));
  for (size_t i = 0; i + 1 < used; i += 2) {
    float t = 0.f;
    RBWS_HIP(hipEventElapsedTime(&t, pool[i], pool[i + 1]));
    ms[kind[i / 2]] += t;
    count[kind[i / 2]] += 1;
  }
  used = 0;
  kind.clear();
}

double wall_clock_khz(int device) {
  int khz = 0;
  RBWS_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
  return (double)khz;
}

// ---------------------------------------------------------------------------
// face-class coefficient tables per solve: kappa = pairwise corner sum * 2^-t
// ---------------------------------------------------------------------------
__global__ void k_kappa(const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                        const double* __restrict__ theta, const uint8_t* const* ncorner,
                        const uint8_t* const* thidx, double* __restrict__ kap64,
                        float* __restrict__ kap32) {
  const int b = blockIdx.x;
  const SolveDev S = sd[b];
  const GridDev& g = pd[S.prob].g;
  const uint8_t* nc = ncorner[S.prob];
  const uint8_t* ti = thidx[S.prob];
  const double* th = theta + (long long)b * kMaxQ;
  const int tot = g.ndir * g.nclass;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int cls = e % g.nclass;
    const uint8_t* id = ti + (long long)e * 8;
    double v;
    switch (nc[cls]) {
      case 1: v = th[id[0]]; break;
      case 2: v = (th[id[0]] + th[id[1]]) * 0.5; break;
      case 4: v = ((th[id[0]] + th[id[1]]) + (th[id[2]] + th[id[3]])) * 0.25; break;
      default:
        v = (((th[id[0]] + th[id[1]]) + (th[id[2]] + th[id[3]])) +
             ((th[id[4]] + th[id[5]]) + (th[id[6]] + th[id[7]]))) * 0.125;
    }
    kap64[S.kap_off + e] = v;
    kap32[S.kap_off + e] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// residual evaluations over (solve, tile) work items: RESID r = f - A x (with
// ||r||^2, r.P(r), ||f||^2 on the first pass), RNORM the same norms only.
// These run a few times per solve; they read neighbours through the caches.
// ---------------------------------------------------------------------------
template <int OP>
__device__ __forceinline__ void k_sweep64_item(int item, const int2* __restrict__ items,
                                                 const SolveDev* __restrict__ sd,
                                                 const ProbDev* __restrict__ pd,
                                                 const CgState* __restrict__ st,
                                                 const double* __restrict__ kap,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 CrAcc* __restrict__ part) {
  extern __shared__ double kl[];
  __shared__ CrAcc red[4];
  __shared__ int zk[kZkLen];
  __syncthreads();  // LDS of the previous item is free
  const int2 it = items[item];
  const int b = it.x, tile = it.y;
  if (OP == OP_AP && st[b].mode != MODE_RESID) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const GridDev& g = P.g;
  const int ntab = g.ndir * g.nclass;
  QuadGeo G;
  quad_geo(G, P, tile);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) kl[e] = kap[S.kap_off + e];
  zk_stage(zk, g, G);
  __syncthreads();
  const int prec = OP == OP_AP ? st[b].prec : 0, first = OP == OP_AP ? st[b].first : 1;
  const int n = g.n;
  CrAcc a0 = cr_zero(), a1 = cr_zero(), a2 = cr_zero();
  double* X = x + S.off;
  double* R = r + S.off;
  for (int k = G.kb; k <= G.ke; k++) {
    const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (e >= G.nv) continue;
      const int i = G.i + e, j = G.j;
      double kk[6];
      quad_kappa<double>(G, kl, e, czn, czm, czp, kk);
      const double dg = diag6(kk);
      const long long c = vidx(n, i, j, k);
      const double q = stencil(kk, dg, X, c, n, i, j, k);
      const double f = fval(P, S, i, j, k);
      const double rv = f - q;
      cr_add_prod(a0, rv, rv);
      if (first) cr_add_prod(a2, f, f);
      if (OP == OP_AP) {
        R[c] = rv;
        if (prec) cr_add_prod(a1, rv, rv / dg);
      }
    }
  }
  CrAcc* out = part + (long long)item * kSlots;
  a0 = cr_block_reduce(a0, red);
  if (threadIdx.x == 0) out[0] = a0;
  if (OP == OP_AP && prec) {
    a1 = cr_block_reduce(a1, red);
    if (threadIdx.x == 0) out[1] = a1;
  }
  if (first) {
    a2 = cr_block_reduce(a2, red);
    if (threadIdx.x == 0) out[2] = a2;
  }
}

template <int OP>
__global__ __launch_bounds__(256) void k_sweep64(const int2* __restrict__ items, const int* __restrict__ list,
                                                 const int* __restrict__ cnt, int nitems,
                                                 const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                 const CgState* __restrict__ st, const double* __restrict__ kap,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 CrAcc* __restrict__ part) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step)
    k_sweep64_item<OP>(list ? list[w] : w, items, sd, pd, st, kap, x, r, part);
}

// ---------------------------------------------------------------------------
// the iteration sweeps of the FP64 path (fast.hpp)
// ---------------------------------------------------------------------------
template <bool VEC, int OP>
__device__ __forceinline__ void k_fast64_item(int item, const int2* __restrict__ items,
                                                const SolveDev* __restrict__ sd,
                                                const ProbDev* __restrict__ pd,
                                                const CgState* __restrict__ st,
                                                const double* __restrict__ kap, double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ p0,
                                                double* __restrict__ p1, CrAcc* __restrict__ part,
                                                int ktab) {
  extern __shared__ __align__(16) double smem[];
  __shared__ CrAcc red[4];
  __shared__ int zk[kZkLen];
  __syncthreads();  // LDS of the previous item is free
  const int2 it = items[item];
  const int b = it.x;
  const CgState& s = st[b];
  if (s.mode != MODE_ITER) return;
  if (OP == FOP_UP2 && s.skip2) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const int ntab = P.g.ndir * P.g.nclass;
  double* kt = smem;
  QuadGeo G;
  quad_geo(G, P, it.y);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) kt[e] = kap[S.kap_off + e];
  zk_stage(zk, P.g, G);
  __syncthreads();
  const int par = s.k & 1;
  const double* Pold = (par ? p1 : p0) + S.off;
  double* Pn = (par ? p0 : p1) + S.off;
  DotAcc<double> a0, a1;
  a0.zero();
  a1.zero();
  fast_body<double, VEC, OP>(G, P.g, kt, smem + ktab, r + S.off, r + S.off, Pold, Pn, x + S.off, s.alpha,
                             s.beta, s.restart, s.prec, 0, a0, a1);
  CrAcc* out = part + (long long)item * kSlots;
  CrAcc t = cr_block_reduce(a0.a, red);
  if (threadIdx.x == 0) out[0] = t;
  if (OP == FOP_UP2 && s.prec) {
    t = cr_block_reduce(a1.a, red);
    if (threadIdx.x == 0) out[1] = t;
  }
}

template <bool VEC, int OP>
__global__ __launch_bounds__(256) void k_fast64(const int2* __restrict__ items, const int* __restrict__ list,
                                                const int* __restrict__ cnt, int nitems,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const CgState* __restrict__ st, const double* __restrict__ kap,
                                                double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ p0, double* __restrict__ p1,
                                                CrAcc* __restrict__ part, int ktab) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step)
    k_fast64_item<VEC, OP>(list ? list[w] : w, items, sd, pd, st, kap, x, r, p0, p1, part, ktab);
}

// ---------------------------------------------------------------------------
// per-solve finalisation (one workgroup per solve)
// ---------------------------------------------------------------------------
struct FinShared {
  CrAcc red[4];
  XAcc xa;
  uint32_t dig[XA_WORDS];
  double val;
  int ok, flag, slot;
};

// exact recomputation of one inner product of solve b (workgroup-cooperative)
__device__ double exact_solve_dot(FinShared& sh, int which, const ProbDev& P, const SolveDev& S,
                                  const double* kap, const double* x, const double* r,
                                  const double* p) {
  const GridDev& g = P.g;
  const int n = g.n;
  __syncthreads();
  xa_clear(&sh.xa);
  __syncthreads();
  const double* X = x + S.off;
  const double* R = r + S.off;
  const double* Pv = p + S.off;
  const double* kt = kap + S.kap_off;
  for (long long c = threadIdx.x; c < g.ndof; c += blockDim.x) {
    const int i = (int)(c % n) + 1, j = (int)((c / n) % n) + 1, k = (int)(c / ((long long)n * n)) + 1;
    if (which == DOT_PAP) {
      double kk[6];
      point_kappa(g, kt, i, j, k, kk);
      xa_add_prod(&sh.xa, Pv[c], stencil(kk, diag6(kk), Pv, c, n, i, j, k));
    } else if (which == DOT_RR) {
      xa_add_prod(&sh.xa, R[c], R[c]);
    } else if (which == DOT_RSV) {
      xa_add_prod(&sh.xa, R[c], Pv[c]);
    } else if (which == DOT_RESID) {
      double kk[6];
      point_kappa(g, kt, i, j, k, kk);
      const double rv = fval(P, S, i, j, k) - stencil(kk, diag6(kk), X, c, n, i, j, k);
      xa_add_prod(&sh.xa, rv, rv);
    } else if (which == DOT_RS) {
      double kk[6];
      point_kappa(g, kt, i, j, k, kk);
      xa_add_prod(&sh.xa, R[c], R[c] / diag6(kk));
    } else {
      const double f = fval(P, S, i, j, k);
      xa_add_prod(&sh.xa, f, f);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.val = xa_round(&sh.xa, sh.dig);
  __syncthreads();
  return sh.val;
}

// reduce slot `slot` of the solve's partials; fall back to the exact path
__device__ double solve_dot(FinShared& sh, int slot, int which, const ProbDev& P, const SolveDev& S,
                            const double* kap, const double* x, const double* r, const double* p,
                            const CrAcc* part, int force_exact) {
  CrAcc a = cr_zero();
  for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x)
    a = cr_combine(a, part[(long long)(S.item0 + t) * kSlots + slot]);
  a = cr_block_reduce(a, sh.red);
  if (threadIdx.x == 0) {
    double v = 0.0;
    sh.ok = (!force_exact && cr_finalize(a, &v)) ? 1 : 0;
    sh.val = v;
  }
  __syncthreads();
  const int ok = sh.ok;
  const double v = sh.val;
  __syncthreads();
  if (ok) return v;
  if (threadIdx.x == 0) atomicAdd(&g_fallback_solver, 1ull);
  return exact_solve_dot(sh, which, P, S, kap, x, r, p);
}

__device__ __forceinline__ void mark_done(CgState& s, int status, int* active) {
  s.status = status;
  s.mode = MODE_DONE;
  s.t_done = wall_clock64();
  atomicSub(active, 1);
}

__global__ __launch_bounds__(256) void k_fin1(const SolveDev* __restrict__ sd,
                                              const ProbDev* __restrict__ pd, CgState* st,
                                              const double* __restrict__ kap, const double* x,
                                              const double* r, const double* p, const double* p1,
                                              const CrAcc* __restrict__ part, int* active,
                                              int force_exact, Lists L) {
  __shared__ FinShared sh;
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) {  // the ap and res sweeps and the last V-cycle are done
    L.cnt[WL_AP] = 0;
    L.cnt[WL_RES] = 0;
    for (int q = 0; q < WL_MAXPROB; q++) L.cnt[WL_MG + q] = 0;
  }
  const int mode = st[b].mode;
  if (mode == MODE_DONE) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  CgState s = st[b];
  if (mode == MODE_ITER) {
    const double* pn = (s.k & 1) ? p : p1;  // the buffer this iteration's AP wrote
    const double g = solve_dot(sh, 0, DOT_PAP, P, S, kap, x, r, pn, part, force_exact);
    if (threadIdx.x == 0) {
      if (!__builtin_isfinite(g)) mark_done(s, RBWS_SOLVE_NAN, active);
      else if (!(g > 0.0)) mark_done(s, RBWS_SOLVE_BREAKDOWN, active);
      else s.alpha = s.rho / g;
      st[b] = s;
      sh.flag = s.mode == MODE_ITER && !s.skip2;
    }
    __syncthreads();
    if (sh.flag) list_push(L.up, L.cnt + WL_UP, S.item0, S.ntiles, &sh.slot);
    return;
  }
  // residual evaluation: the initial residual or a true-residual confirmation
  const double rr = solve_dot(sh, 0, DOT_RR, P, S, kap, x, r, p, part, force_exact);
  const double rs = s.prec ? solve_dot(sh, 1, DOT_RS, P, S, kap, x, r, p, part, force_exact) : rr;
  double ff = s.ff;
  if (s.first) ff = solve_dot(sh, 2, DOT_FF, P, S, kap, x, r, p, part, force_exact);
  if (threadIdx.x == 0) {
    if (s.first) {
      s.ff = ff;
      s.thr = s.tol2 * ff;
      s.init_rr = rr;
      s.first = 0;
    }
    s.rr = rr;
    if (!__builtin_isfinite(rr)) mark_done(s, RBWS_SOLVE_NAN, active);
    else if (rr <= s.thr) mark_done(s, RBWS_SOLVE_CONVERGED, active);
    else if (s.k >= s.maxit) mark_done(s, RBWS_SOLVE_MAXITER, active);
    else {
      if (!s.mg) s.rho = rs;  // with a V-cycle, rho = r^T s follows the preconditioner step
      s.restart = 1;
      s.mode = MODE_ITER;
      s.skip2 = 1;  // no update this round: the next round starts with p = s
    }
    st[b] = s;
  }
}

__global__ __launch_bounds__(256) void k_fin2(const SolveDev* __restrict__ sd,
                                              const ProbDev* __restrict__ pd, CgState* st,
                                              const double* __restrict__ kap, const double* x,
                                              const double* r, const double* p,
                                              const CrAcc* __restrict__ part, int* active,
                                              int force_exact, Lists L, int* need) {
  __shared__ FinShared sh;
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) L.cnt[WL_UP] = 0;  // the up sweep of this round is done
  const int mode = st[b].mode;
  if (need && threadIdx.x == 0) need[b] = 0;
  if (mode == MODE_DONE) return;
  const SolveDev S = sd[b];
  if (mode == MODE_RESID) {
    list_push(L.res, L.cnt + WL_RES, S.item0, S.ntiles, &sh.slot);
    return;
  }
  CgState s = st[b];
  if (s.skip2) {
    if (threadIdx.x == 0) {
      st[b].skip2 = 0;
      if (need) {  // the V-cycle on the (re)started residual
        need[b] = 1;
        st[b].nvc += 1;
        const int q = sd[b].prob;
        L.mg[L.cnt[WL_SEG + q] + atomicAdd(&L.cnt[WL_MG + q], 1)] = L.gidx[b];
      }
    }
    list_push(L.ap, L.cnt + WL_AP, S.item0, S.ntiles, &sh.slot);
    return;
  }
  const ProbDev& P = pd[S.prob];
  const double rr = solve_dot(sh, 0, DOT_RR, P, S, kap, x, r, p, part, force_exact);
  const double rs = s.prec ? solve_dot(sh, 1, DOT_RS, P, S, kap, x, r, p, part, force_exact) : rr;
  if (threadIdx.x == 0) {
    s.k += 1;
    s.rr = rr;
    if (!__builtin_isfinite(rr)) mark_done(s, RBWS_SOLVE_NAN, active);
    else if (rr <= s.thr) {  // confirm with the true residual next round
      s.mode = MODE_RESID;
      s.extra += 1;
    } else if (s.k >= s.maxit) mark_done(s, RBWS_SOLVE_MAXITER, active);
    else if (s.mg) {
      s.restart = 0;  // beta and rho follow the V-cycle (k_fin_mg)
      s.nvc += 1;
      need[b] = 1;
      L.mg[L.cnt[WL_SEG + S.prob] + atomicAdd(&L.cnt[WL_MG + S.prob], 1)] = L.gidx[b];
    } else {
      s.beta = rs / s.rho;
      s.rho = rs;
      s.restart = 0;
    }
    st[b] = s;
    sh.flag = s.mode;
  }
  __syncthreads();
  const int nm = sh.flag;
  if (nm == MODE_ITER) list_push(L.ap, L.cnt + WL_AP, S.item0, S.ntiles, &sh.slot);
  else if (nm == MODE_RESID) list_push(L.res, L.cnt + WL_RES, S.item0, S.ntiles, &sh.slot);
}

// r^T s over the tiles of the solves on a list (s from the V-cycle), into partial slot 1
__device__ __forceinline__ void k_dot_rs_item(int item, const int2* __restrict__ items,
                                              const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                              const double* __restrict__ r, const double* __restrict__ sv,
                                              CrAcc* __restrict__ part) {
  __shared__ CrAcc red[4];
  __syncthreads();
  const int2 it = items[item];
  const SolveDev S = sd[it.x];
  const ProbDev& P = pd[S.prob];
  QuadGeo G;
  quad_geo(G, P, it.y);
  const int n = P.g.n;
  CrAcc a = cr_zero();
  for (int k = G.kb; k <= G.ke; k++) {
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (e >= G.nv) continue;
      const long long c = S.off + vidx(n, G.i + e, G.j, k);
      cr_add_prod(a, r[c], sv[c]);
    }
  }
  a = cr_block_reduce(a, red);
  if (threadIdx.x == 0) part[(long long)item * kSlots + 1] = a;
}

__global__ __launch_bounds__(256) void k_dot_rs(const int2* __restrict__ items, const int* __restrict__ list,
                                                const int* __restrict__ cnt, int nitems,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const double* __restrict__ r, const double* __restrict__ sv,
                                                CrAcc* __restrict__ part) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step) k_dot_rs_item(list ? list[w] : w, items, sd, pd, r, sv, part);
}

// after the V-cycle: rho' = r^T s, then beta = rho' / rho (or a restart: p = s)
__global__ __launch_bounds__(256) void k_fin_mg(const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                CgState* st, const double* __restrict__ kap, const double* x,
                                                const double* r, const double* sv,
                                                const CrAcc* __restrict__ part, const int* __restrict__ need,
                                                int force_exact) {
  __shared__ FinShared sh;
  const int b = blockIdx.x;
  if (!need[b]) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const double rs = solve_dot(sh, 1, DOT_RSV, P, S, kap, x, r, sv, part, force_exact);
  if (threadIdx.x == 0) {
    CgState s = st[b];
    if (!s.restart) s.beta = rs / s.rho;
    s.rho = rs;
    st[b] = s;
  }
}

__global__ __launch_bounds__(256) void k_fin_rnorm(const SolveDev* __restrict__ sd,
                                                   const ProbDev* __restrict__ pd,
                                                   const double* __restrict__ kap, const double* x,
                                                   const CrAcc* __restrict__ part, double* out,
                                                   int force_exact) {
  __shared__ FinShared sh;
  const int b = blockIdx.x;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const double rr = solve_dot(sh, 0, DOT_RESID, P, S, kap, x, nullptr, nullptr, part, force_exact);
  const double ff = solve_dot(sh, 2, DOT_FF, P, S, kap, x, nullptr, nullptr, part, force_exact);
  if (threadIdx.x == 0) {
    out[3 * b + 0] = sqrt(rr / ff);
    out[3 * b + 1] = rr;
    out[3 * b + 2] = ff;
  }
}

// ---------------------------------------------------------------------------
// y = A x (FP64 or FP32) for every solve of the batch
// ---------------------------------------------------------------------------
template <typename T, bool VEC>
__device__ __forceinline__ void k_spmv_item(int item, const int2* __restrict__ items,
                                              const SolveDev* __restrict__ sd,
                                              const ProbDev* __restrict__ pd,
                                              const T* __restrict__ kap, const T* __restrict__ x,
                                              T* __restrict__ y, int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  __shared__ int zk[kZkLen];
  __syncthreads();  // LDS of the previous item is free
  const int2 it = items[item];
  const SolveDev S = sd[it.x];
  const ProbDev& P = pd[S.prob];
  const int ntab = P.g.ndir * P.g.nclass;
  QuadGeo G;
  quad_geo(G, P, it.y);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) smem[e] = kap[S.kap_off + e];
  zk_stage(zk, P.g, G);
  __syncthreads();
  DotAcc<T> a0, a1;
  fast_body<T, VEC, FOP_SPMV>(G, P.g, smem, smem + ktab, nullptr, nullptr, nullptr,
                              const_cast<T*>(x) + S.off, y + S.off, T(0), T(0), 0, 0, 0, a0, a1);
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_spmv(const int2* __restrict__ items, int nitems,
                                              const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                              const T* __restrict__ kap, const T* __restrict__ x,
                                              T* __restrict__ y, int ktab) {
  const WorkRange R = work_range(nitems);
  for (int w = R.w; w < R.w1; w += R.step) k_spmv_item<T, VEC>(w, items, sd, pd, kap, x, y, ktab);
}

// ---------------------------------------------------------------------------
// generic correctly rounded dots (for the ABI and the reduced-basis code)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ x,
                                                  const double* __restrict__ y, long long len,
                                                  int per_block, CrAcc* __restrict__ part) {
  __shared__ CrAcc red[4];
  const int v = blockIdx.y;
  const long long beg = (long long)blockIdx.x * per_block;
  const long long end = min(len, beg + per_block);
  const double* X = x + (long long)v * len;
  const double* Y = y + (long long)v * len;
  CrAcc a = cr_zero();
  for (long long c = beg + threadIdx.x; c < end; c += blockDim.x) cr_add_prod(a, X[c], Y[c]);
  a = cr_block_reduce(a, red);
  if (threadIdx.x == 0) part[(long long)v * gridDim.x + blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void k_dot_fin(const double* __restrict__ x,
                                                 const double* __restrict__ y, long long len,
                                                 int nparts, const CrAcc* __restrict__ part,
                                                 double* __restrict__ out, int force_exact) {
  __shared__ FinShared sh;
  const int v = blockIdx.x;
  CrAcc a = cr_zero();
  for (int t = threadIdx.x; t < nparts; t += blockDim.x) a = cr_combine(a, part[(long long)v * nparts + t]);
  a = cr_block_reduce(a, sh.red);
  if (threadIdx.x == 0) {
    double r = 0.0;
    sh.ok = (!force_exact && cr_finalize(a, &r)) ? 1 : 0;
    sh.val = r;
  }
  __syncthreads();
  if (sh.ok) {
    if (threadIdx.x == 0) out[v] = sh.val;
    return;
  }
  if (threadIdx.x == 0) atomicAdd(&g_fallback_solver, 1ull);
  __syncthreads();
  xa_clear(&sh.xa);
  __syncthreads();
  const double* X = x + (long long)v * len;
  const double* Y = y + (long long)v * len;
  for (long long c = threadIdx.x; c < len; c += blockDim.x) xa_add_prod(&sh.xa, X[c], Y[c]);
  __syncthreads();
  if (threadIdx.x == 0) out[v] = xa_round(&sh.xa, sh.dig);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void batch_setup(Batch& B, const std::vector<const Problem*>& probs, const int* prob_of, int nsolve,
                 const double* mu, int p, hipStream_t s, const double* theta_override, bool internal) {
  RBWS_REQUIRE(!probs.empty(), RBWS_EINVAL, "no problem");
  B.device = probs[0]->device;
  RBWS_HIP(hipSetDevice(B.device));
  B.probs = probs;
  B.nprob = (int)probs.size();
  B.nsolve = nsolve;
  B.pd_h.assign(B.nprob, ProbDev{});
  std::vector<const uint8_t*> ncp(B.nprob), thp(B.nprob);
  for (int q = 0; q < B.nprob; q++) {
    const Problem* P = probs[q];
    RBWS_REQUIRE(P->device == B.device, RBWS_EINVAL, "problems of one batch must share a device");
    RBWS_REQUIRE(P->p == p, RBWS_EINVAL, "problems of one batch must share p");
    ProbDev& d = B.pd_h[q];
    d.g = P->grid;
    long long cnt = 0;
    for (int b = 0; b < nsolve; b++) cnt += (prob_of ? prob_of[b] : 0) == q;
    choose_tile(P->n, cnt, &d.TX, &d.TY, &d.TZ, internal);
    RBWS_REQUIRE(d.TZ >= 1 && d.TZ <= kTzMax, RBWS_EINVAL, "tile depth out of range");
    d.ntx = (P->n + d.TX - 1) / d.TX;
    d.nty = (P->n + d.TY - 1) / d.TY;
    d.ntz = (P->n + d.TZ - 1) / d.TZ;
    d.ntiles = d.ntx * d.nty * d.ntz;
    d.f_kind = P->desc.f_kind;
    d.h = 1.0 / (P->n + 1);
    d.h2 = d.h * d.h;
    d.gw = P->desc.gauss_width;
    ncp[q] = P->ct_ncorner_dev;
    thp[q] = P->ct_theta_dev;
  }
  B.sd_h.assign(nsolve, SolveDev{});
  B.items_h.clear();
  std::vector<double>& theta = B.theta_h;  // kept: the copy below is asynchronous
  theta.assign((size_t)std::max(nsolve, 1) * kMaxQ, 0.0);
  long long off = 0, koff = 0;
  B.kap_max = 0;
  for (int b = 0; b < nsolve; b++) {
    int q = prob_of ? prob_of[b] : 0;
    RBWS_REQUIRE(q >= 0 && q < B.nprob, RBWS_EINVAL, "problem_of entry out of range");
    const Problem* P = probs[q];
    const ProbDev& d = B.pd_h[q];
    SolveDev& S = B.sd_h[b];
    S.prob = q;
    S.ntiles = d.ntiles;
    S.item0 = (int)B.items_h.size();
    S.off = off;
    S.kap_off = koff;
    if (theta_override) {
      for (int t = 0; t < P->Q; t++) theta[(size_t)b * kMaxQ + t] = theta_override[(size_t)b * P->Q + t];
    } else {
      const double* m = mu + (long long)b * p;
      for (int t = 0; t < p; t++)
        RBWS_REQUIRE(std::isfinite(m[t]), RBWS_EINVAL, "mu must be finite");
      if (P->desc.f_kind == RBWS_F_GAUSS) {
        S.x0[0] = m[24];
        S.x0[1] = m[25];
        S.x0[2] = m[26];
      }
      theta_host(*P, m, &theta[(size_t)b * kMaxQ]);
    }
    off += P->ndof;
    int tab = P->grid.ndir * P->grid.nclass;
    koff += tab;
    B.kap_max = std::max(B.kap_max, tab);
    for (int t = 0; t < d.ntiles; t++) B.items_h.push_back(make_int2(b, t));
  }
  B.total = off;
  B.kap_total = koff;
  B.nitems = (int)B.items_h.size();
  B.vec = true;
  for (const Problem* P : probs) B.vec = B.vec && (P->n % 4 == 0);
  RBWS_HIP(hipMemcpyAsync(B.pd.get(sizeof(ProbDev) * B.nprob, B.device), B.pd_h.data(),
                          sizeof(ProbDev) * B.nprob, hipMemcpyHostToDevice, s));
  if (nsolve > 0) {
    RBWS_HIP(hipMemcpyAsync(B.sd.get(sizeof(SolveDev) * nsolve, B.device), B.sd_h.data(),
                            sizeof(SolveDev) * nsolve, hipMemcpyHostToDevice, s));
    RBWS_HIP(hipMemcpyAsync(B.items.get(sizeof(int2) * B.nitems, B.device), B.items_h.data(),
                            sizeof(int2) * B.nitems, hipMemcpyHostToDevice, s));
    RBWS_HIP(hipMemcpyAsync(B.theta.get(sizeof(double) * theta.size(), B.device), theta.data(),
                            sizeof(double) * theta.size(), hipMemcpyHostToDevice, s));
  }
  RBWS_HIP(hipMemcpyAsync(B.ncorner.get(sizeof(void*) * B.nprob, B.device), ncp.data(),
                          sizeof(void*) * B.nprob, hipMemcpyHostToDevice, s));
  RBWS_HIP(hipMemcpyAsync(B.thidx.get(sizeof(void*) * B.nprob, B.device), thp.data(),
                          sizeof(void*) * B.nprob, hipMemcpyHostToDevice, s));
  B.kap64.get(sizeof(double) * std::max<long long>(B.kap_total, 1), B.device);
  B.kap32.get(sizeof(float) * std::max<long long>(B.kap_total, 1), B.device);
  if (nsolve > 0) {
    hipLaunchKernelGGL(k_kappa, dim3(nsolve), dim3(256), 0, s, (const SolveDev*)B.sd.ptr,
                       (const ProbDev*)B.pd.ptr, (const double*)B.theta.ptr,
                       (const uint8_t* const*)B.ncorner.ptr, (const uint8_t* const*)B.thidx.ptr,
                       (double*)B.kap64.ptr, (float*)B.kap32.ptr);
    RBWS_HIP(hipGetLastError());
  }
  if (!B.active_host) RBWS_HIP(hipHostMalloc((void**)&B.active_host, 64, hipHostMallocDefault));
}

void cg_fp64_run(Batch& B, const CgOpts& o, hipStream_t s) {
  RBWS_HIP(hipSetDevice(B.device));
  const int ns = B.nsolve;
  if (ns == 0) return;
  std::vector<CgState> init(ns);
  for (int b = 0; b < ns; b++) {
    CgState& c = init[b];
    std::memset(&c, 0, sizeof c);
    c.tol2 = o.tol * o.tol;
    c.status = -1;
    c.mode = MODE_RESID;
    c.restart = 1;
    c.maxit = o.maxit;
    c.prec = o.prec;
    c.first = 1;
  }
  const bool mg = o.prec == RBWS_PREC_MG;
  if (mg)
    for (CgState& c : init) {
      c.prec = 0;  // the sweeps form ||r||^2 only; s and r^T s come from the V-cycle
      c.mg = 1;
    }
  CgState* st = (CgState*)B.state.get(sizeof(CgState) * ns, B.device);
  RBWS_HIP(hipMemcpyAsync(st, init.data(), sizeof(CgState) * ns, hipMemcpyHostToDevice, s));
  int* active = (int*)B.active.get(sizeof(int), B.device);
  RBWS_HIP(hipMemcpyAsync(active, &ns, sizeof(int), hipMemcpyHostToDevice, s));
  CrAcc* part = (CrAcc*)B.part.get(sizeof(CrAcc) * kSlots * B.nitems, B.device);
  double* x = (double*)B.x.ptr;
  double* r = (double*)B.r.get(sizeof(double) * B.total, B.device);
  double* p = (double*)B.p.get(sizeof(double) * B.total, B.device);
  RBWS_REQUIRE(x != nullptr && B.x.bytes >= sizeof(double) * B.total, RBWS_ESTATE, "initial guess missing");
  const int2* items = (const int2*)B.items.ptr;
  const SolveDev* sd = (const SolveDev*)B.sd.ptr;
  const ProbDev* pd = (const ProbDev*)B.pd.ptr;
  const double* kap = (const double*)B.kap64.ptr;
  const size_t lds = sizeof(double) * B.kap_max;
  const int fe = (o.flags & RBWS_FLAG_FORCE_EXACT_DOTS) ? 1 : 0;
  const int check = o.check_every > 0 ? o.check_every : 4;
  const long long max_rounds = 2LL * o.maxit + 16;
  double* p1 = (double*)B.p2.get(sizeof(double) * B.total, B.device);
  const int ni = B.nitems;
  const int ktab = (B.kap_max + 3) & ~3;
  const size_t lds_fast = sizeof(double) * (ktab + 2 * QPLANE);
  auto ap = B.vec ? k_fast64<true, FOP_AP> : k_fast64<false, FOP_AP>;
  auto up = B.vec ? k_fast64<true, FOP_UP2> : k_fast64<false, FOP_UP2>;
  auto res = k_sweep64<OP_AP>;
  const unsigned g_ap = persistent_grid((const void*)ap, lds_fast, ni, B.device);
  const unsigned g_up = persistent_grid((const void*)up, lds_fast, ni, B.device);
  const unsigned g_res = persistent_grid((const void*)res, lds, ni, B.device);
  const Lists L = lists_init(B, s);
  MgRun* mgr = nullptr;
  double* sv = r;  // the vector the direction update reads: r (P = I, Jacobi in-kernel) or s
  int* need = nullptr;
  if (mg) {
    mgr = mg_prepare(B, o.mg_nu, o.mg_omega, false, s);
    sv = (double*)B.sv.get(sizeof(double) * B.total, B.device);
    need = (int*)B.need.get(sizeof(int) * ns, B.device);
    std::vector<int> z(ns, 0);
    RBWS_HIP(hipMemcpyAsync(need, z.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    RBWS_HIP(hipStreamSynchronize(s));
  }
  const unsigned g_dot = mg ? persistent_grid((const void*)k_dot_rs, 0, ni, B.device) : 0;
  KernelTimer& kt = ktimer();
  const bool graph = !(o.flags & RBWS_FLAG_NO_GRAPH) && !kt.on;
  run_rounds(B, active, max_rounds, check, graph, s, [&](hipStream_t q) {
    kt.begin(q, KK_AP);
    hipLaunchKernelGGL(ap, dim3(g_ap), dim3(256), lds_fast, q, items, L.ap, L.cnt + WL_AP, ni, sd, pd, st, kap,
                       x, sv, p, p1, part, ktab);
    kt.end(q);
    kt.begin(q, KK_RESID);
    hipLaunchKernelGGL(res, dim3(g_res), dim3(256), lds, q, items, L.res, L.cnt + WL_RES, ni, sd, pd, st, kap, x,
                       r, part);
    kt.end(q);
    kt.begin(q, KK_FIN1);
    hipLaunchKernelGGL(k_fin1, dim3(ns), dim3(256), 0, q, sd, pd, st, kap, x, r, p, p1, part, active, fe, L);
    kt.end(q);
    kt.begin(q, KK_UP2);
    hipLaunchKernelGGL(up, dim3(g_up), dim3(256), lds_fast, q, items, L.up, L.cnt + WL_UP, ni, sd, pd, st, kap,
                       x, r, p, p1, part, ktab);
    kt.end(q);
    kt.begin(q, KK_FIN2);
    hipLaunchKernelGGL(k_fin2, dim3(ns), dim3(256), 0, q, sd, pd, st, kap, x, r, p, part, active, fe, L, need);
    kt.end(q);
    if (mg) {
      const bool fused = mg_apply(mgr, B, r, sv, L, part, q);  // times its own kernels
      kt.begin(q, KK_MG);
      if (!fused)
        hipLaunchKernelGGL(k_dot_rs, dim3(g_dot), dim3(256), 0, q, items, (const int*)L.ap,
                           (const int*)(L.cnt + WL_AP), ni, sd, pd, (const double*)r, (const double*)sv, part);
      hipLaunchKernelGGL(k_fin_mg, dim3(ns), dim3(256), 0, q, sd, pd, st, kap, (const double*)x, (const double*)r,
                         (const double*)sv, (const CrAcc*)part, (const int*)need, fe);
      kt.end(q);
    }
  });
}

void resid_norms(Batch& B, const double* x, double* rel, double* rr, double* ff, int force_exact,
                 hipStream_t s) {
  RBWS_HIP(hipSetDevice(B.device));
  const int ns = B.nsolve;
  if (ns == 0) return;
  CrAcc* part = (CrAcc*)B.part.get(sizeof(CrAcc) * kSlots * B.nitems, B.device);
  // the sweep reads the solve mode from a state array; any mode runs OP_RNORM
  CgState* st = (CgState*)B.state.get(sizeof(CgState) * ns, B.device);
  RBWS_SCRATCH(outb);
  double* o = (double*)outb.get(sizeof(double) * 3 * ns, B.device);
  const size_t lds = sizeof(double) * B.kap_max;
  const unsigned grid = persistent_grid((const void*)k_sweep64<OP_RNORM>, lds, B.nitems, B.device);
  hipLaunchKernelGGL(k_sweep64<OP_RNORM>, dim3(grid), dim3(256), lds, s, (const int2*)B.items.ptr,
                     (const int*)nullptr, (const int*)nullptr, B.nitems, (const SolveDev*)B.sd.ptr,
                     (const ProbDev*)B.pd.ptr, st, (const double*)B.kap64.ptr, (double*)x, nullptr, part);
  hipLaunchKernelGGL(k_fin_rnorm, dim3(ns), dim3(256), 0, s, (const SolveDev*)B.sd.ptr,
                     (const ProbDev*)B.pd.ptr, (const double*)B.kap64.ptr, x, part, o, force_exact);
  RBWS_HIP(hipGetLastError());
  std::vector<double> h(3 * (size_t)ns);
  RBWS_HIP(hipMemcpyAsync(h.data(), o, sizeof(double) * 3 * ns, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < ns; b++) {
    if (rel) rel[b] = h[3 * b];
    if (rr) rr[b] = h[3 * b + 1];
    if (ff) ff[b] = h[3 * b + 2];
  }
}

void states_to_host(Batch& B, std::vector<CgState>& out, hipStream_t s) {
  out.resize(B.nsolve);
  if (B.nsolve == 0) return;
  RBWS_HIP(hipMemcpyAsync(out.data(), B.state.ptr, sizeof(CgState) * B.nsolve, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
}

void spmv_batch(Batch& B, const void* x, void* y, bool fp32, hipStream_t s) {
  RBWS_HIP(hipSetDevice(B.device));
  if (B.nsolve == 0) return;
  const int ktab = (B.kap_max + 3) & ~3;
  const int2* it = (const int2*)B.items.ptr;
  const SolveDev* sd = (const SolveDev*)B.sd.ptr;
  const ProbDev* pd = (const ProbDev*)B.pd.ptr;
  ktimer().begin(s, KK_SPMV);
  if (fp32) {
    auto k = B.vec ? k_spmv<float, true> : k_spmv<float, false>;
    const size_t lds = sizeof(float) * (ktab + 2 * QPLANE);
    hipLaunchKernelGGL(k, dim3(persistent_grid((const void*)k, lds, B.nitems, B.device)), dim3(256), lds, s, it,
                       B.nitems, sd, pd, (const float*)B.kap32.ptr, (const float*)x, (float*)y, ktab);
  } else {
    auto k = B.vec ? k_spmv<double, true> : k_spmv<double, false>;
    const size_t lds = sizeof(double) * (ktab + 2 * QPLANE);
    hipLaunchKernelGGL(k, dim3(persistent_grid((const void*)k, lds, B.nitems, B.device)), dim3(256), lds, s, it,
                       B.nitems, sd, pd, (const double*)B.kap64.ptr, (const double*)x, (double*)y, ktab);
  }
  ktimer().end(s);
  RBWS_HIP(hipGetLastError());
}

// Elements per partial sum of the dot kernels, and the number of partials of
// one vector of length len.
constexpr int kDotPerBlock = 4096;
static long long dot_parts(long long len) {
  long long nb = std::max<long long>(1, (len + kDotPerBlock - 1) / kDotPerBlock);
  RBWS_REQUIRE(nb < (1LL << 31), RBWS_EINVAL, "vector too long");
  return nb;
}

// The two dot kernels on the stream: partial double-double sums into `pp`
// (nb * count records, every one written), then one correctly rounded value
// per vector pair into the device array `o`.
static void launch_dots(const double* x, const double* y, long long len, int count, long long nb, CrAcc* pp,
                        double* o, int flags, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_part, dim3((unsigned)nb, count), dim3(256), 0, s, x, y, len, kDotPerBlock, pp);
  hipLaunchKernelGGL(k_dot_fin, dim3(count), dim3(256), 0, s, x, y, len, (int)nb, pp, o,
                     (flags & RBWS_FLAG_FORCE_EXACT_DOTS) ? 1 : 0);
  RBWS_HIP(hipGetLastError());
}

void exact_dots(const double* x, const double* y, long long len, int count, double* out_host,
                int flags, hipStream_t s) {
  if (count <= 0) return;
  int dev = 0;
  RBWS_HIP(hipGetDevice(&dev));
  RBWS_SCRATCH(part);
  RBWS_SCRATCH(out);
  const long long nb = dot_parts(len);
  CrAcc* pp = (CrAcc*)part.get(sizeof(CrAcc) * nb * count, dev);
  double* o = (double*)out.get(sizeof(double) * count, dev);
  launch_dots(x, y, len, count, nb, pp, o, flags, s);
  RBWS_HIP(hipMemcpyAsync(out_host, o, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
}

// Plain device copy with 16-byte non-temporal loads and stores: a workgroup
// moves kCopyWords consecutive 16-byte words, each thread four of them with
// all loads issued before the stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyWords = 1024;
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     long long nwords) {
  const long long base = (long long)blockIdx.x * kCopyWords + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const long long i = base + u * 256;
    if (i < nwords) v[u] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const long long i = base + u * 256;
    if (i < nwords) __builtin_nontemporal_store(v[u], dst + i);
  }
}

void stream_copy(const void* src, void* dst, long long bytes, hipStream_t s) {
  const long long nwords = bytes / 16;
  const long long blocks = (nwords + kCopyWords - 1) / kCopyWords;
  RBWS_REQUIRE(blocks < (1LL << 31), RBWS_EINVAL, "copy too large");
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst,
                     nwords);
  RBWS_HIP(hipGetLastError());
}

// Fixed workspace of exact_dots_noalloc: the partial sums of one call.  Each
// GPU the library runs on holds its own copy of this array until the process
// ends.  In host code its name is not a device address: the address on the
// current device comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[RBWS_NOALLOC_SCRATCH_BYTES];

static void* noalloc_scratch(int dev) {
  static std::mutex mu;
  static std::vector<void*> ptr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)ptr.size() <= dev) ptr.resize(dev + 1, nullptr);
  if (!ptr[dev]) {
    void* a = nullptr;
    RBWS_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    RBWS_REQUIRE(a != nullptr, RBWS_EDEVICE, "no device address for the workspace");
    ptr[dev] = a;
  }
  return ptr[dev];
}

void exact_dots_noalloc(const double* x, const double* y, long long len, int count, double* out_dev,
                        int flags, hipStream_t s) {
  if (count <= 0) return;
  int dev = 0;
  RBWS_HIP(hipGetDevice(&dev));
  if (len == 0) {
    fill64(out_dev, count, 0.0, s);
    return;
  }
  const long long nb = dot_parts(len);
  const unsigned long long need = (unsigned long long)sizeof(CrAcc) * (unsigned long long)nb * (unsigned)count;
  RBWS_REQUIRE(need <= RBWS_NOALLOC_SCRATCH_BYTES, RBWS_EINVAL,
               "count * ceil(len / 4096) = " + std::to_string(nb * count) + " partial sums exceed the " +
                   std::to_string(RBWS_NOALLOC_SCRATCH_BYTES / sizeof(CrAcc)) + " the fixed workspace holds");
  CrAcc* pp = (CrAcc*)noalloc_scratch(dev);
  launch_dots(x, y, len, count, nb, pp, out_dev, flags, s);
}

}  // namespace rbws
