// capi.hip -- extern "C" entry points of librbws.so (declared in include/rbws.h).
// Argument checking, error translation and orchestration of the batched solve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mg.hpp"
#include "mlp.hpp"
#include "rb.hpp"

namespace rbws {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

Problem* problem_create(const rbws_problem_desc* d, int device);
void problem_destroy(Problem* P);

__global__ void k_fill64(double* x, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_stamp(unsigned long long* t) { *t = wall_clock64(); }

// x_b <- src_b for the solves with pick[b] != 0 (grid.y = solve)
__global__ void k_pick(double* __restrict__ x, const double* __restrict__ src, const long long* __restrict__ off,
                       const long long* __restrict__ len, const int* __restrict__ pick) {
  const int b = blockIdx.y;
  if (!pick[b]) return;
  const long long o = off[b], n = len[b];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[o + i] = src[o + i];
}

// c[b] = cr[b] (both stride 64) for the solves with pick[b]
__global__ void k_pick_rows(double* __restrict__ c, const double* __restrict__ cr, const int* __restrict__ pick) {
  const int b = blockIdx.x;
  if (pick[b]) c[(long long)b * 64 + threadIdx.x] = cr[(long long)b * 64 + threadIdx.x];
}

void fill64(double* x, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill64, dim3((unsigned)blocks), dim3(256), 0, s, x, n, v);
  RBWS_HIP(hipGetLastError());
}

// stats of all solves of a batch after a run
void collect_stats(Batch& B, unsigned long long t0, const std::vector<int>& init_used, int outer_field_from_extra,
                   rbws_solve_stat* out, hipStream_t s) {
  std::vector<CgState> st;
  states_to_host(B, st, s);
  const double khz = wall_clock_khz(B.device);
  for (int b = 0; b < B.nsolve; b++) {
    rbws_solve_stat& o = out[b];
    std::memset(&o, 0, sizeof o);
    o.iters = st[b].k;
    o.extra_spmv = st[b].extra;
    o.outer_iters = 0;
    (void)outer_field_from_extra;
    o.status = st[b].status < 0 ? RBWS_SOLVE_MAXITER : st[b].status;
    o.init_used = init_used[b];
    o.vcycles = st[b].nvc;
    o.init_rr = st[b].init_rr;
    o.final_rr = st[b].rr;
    o.ff = st[b].ff;
    o.t_done_ms = st[b].t_done > t0 ? (double)(st[b].t_done - t0) / khz : 0.0;
  }
}

// The learned start: c from the networks, u = V c, and the fallback to the
// reduced solve (0: per solve the start with the smaller true residual; 1: the
// RB start where the network's relative residual exceeds the basis's final
// greedy indicator).  `used` receives RBWS_INIT_LEARNED or RBWS_INIT_RB.
template <class Lift>
void learned_start(Batch& B, const std::vector<const Basis*>& bl, const std::vector<Mlp*>& ml,
                   const int* problem_of, const double* mu, int fallback, int fe, bool allow_est, hipStream_t s,
                   Lift lift, std::vector<int>& used) {
  const int ns = B.nsolve, nprob = B.nprob, p = B.probs[0]->p;
  RBWS_SCRATCH(cm_b);
  RBWS_SCRATCH(cr_b);
  RBWS_SCRATCH(rows_b);
  RBWS_SCRATCH(meta_b);
  double* cm = (double*)cm_b.get(sizeof(double) * 64 * ns, B.device);
  double* x = (double*)B.x.ptr;
  for (int q = 0; q < nprob; q++) {
    if (nprob == 1) {
      mlp_predict_dev(ml[0], mu, ns, nullptr, cm, 64, s);
      break;
    }
    std::vector<int> rows;
    std::vector<double> mq;
    for (int b = 0; b < ns; b++)
      if ((problem_of ? problem_of[b] : 0) == q) {
        rows.push_back(b);
        mq.insert(mq.end(), mu + (long long)b * p, mu + (long long)(b + 1) * p);
      }
    if (rows.empty()) continue;
    int* rd = (int*)rows_b.get(sizeof(int) * rows.size(), B.device);
    RBWS_HIP(hipMemcpyAsync(rd, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, s));
    mlp_predict_dev(ml[q], mq.data(), (int)rows.size(), rd, cm, 64, s);
    RBWS_HIP(hipStreamSynchronize(s));  // rows_b is reused by the next problem
  }
  std::vector<double> rel_m(ns), rel_r(ns);
  // strict rule from the residual decomposition: both residual norms in
  // O(Q^2 N^2) per solve, then one lift of the chosen coefficients
  bool est = fallback == 0 && allow_est;
  for (const Basis* b : bl) est = est && b != nullptr && b->est;
  if (est) {
    double* cr = (double*)cr_b.get(sizeof(double) * 64 * ns, B.device);
    RBWS_REQUIRE(rb_coeffs(B, bl, cr, 64, fe, s) == 0, RBWS_ENUMERIC, "reduced matrix not positive definite");
    const int bad = rb_resid_estimate(B, bl, cm, 64, rel_m.data(), s) + rb_resid_estimate(B, bl, cr, 64, rel_r.data(), s);
    if (bad == 0) {
      std::vector<int> pick(ns);
      for (int b = 0; b < ns; b++) pick[b] = (rel_r[b] < rel_m[b] || !(rel_m[b] == rel_m[b])) ? 1 : 0;
      int* pd = (int*)rows_b.get(sizeof(int) * ns, B.device);
      RBWS_HIP(hipMemcpyAsync(pd, pick.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_pick_rows, dim3(ns), dim3(64), 0, s, cm, (const double*)cr, (const int*)pd);
      RBWS_HIP(hipGetLastError());
      lift(cm, x);
      RBWS_HIP(hipStreamSynchronize(s));  // `pick` outlives the copy
      for (int b = 0; b < ns; b++) used[b] = pick[b] ? RBWS_INIT_RB : RBWS_INIT_LEARNED;
      return;
    }
  }
  lift(cm, x);
  resid_norms(B, x, rel_m.data(), nullptr, nullptr, fe, s);
  std::vector<int> pick(ns, 0);
  bool any = false;
  for (int b = 0; b < ns; b++) {
    RBWS_REQUIRE(fallback == 0 || bl[B.sd_h[b].prob]->kind == 0, RBWS_EINVAL,
                 "the cheap fallback rule needs a Galerkin basis (its indicator is a residual norm)");
    const double thr = bl[B.sd_h[b].prob]->final_max;
    const bool need = fallback == 0 || !(rel_m[b] <= thr);
    pick[b] = need ? 1 : 0;
    any = any || need;
  }
  if (any) {
    double* cr = (double*)cr_b.get(sizeof(double) * 64 * ns, B.device);
    RBWS_REQUIRE(rb_coeffs(B, bl, cr, 64, fe, s) == 0, RBWS_ENUMERIC, "reduced matrix not positive definite");
    double* tmp = (double*)B.r.get(sizeof(double) * B.total, B.device);
    lift(cr, tmp);
    if (fallback == 0) {
      resid_norms(B, tmp, rel_r.data(), nullptr, nullptr, fe, s);
      for (int b = 0; b < ns; b++) pick[b] = (rel_r[b] < rel_m[b] || !(rel_m[b] == rel_m[b])) ? 1 : 0;
    }
    std::vector<long long> meta(3 * (size_t)ns);
    for (int b = 0; b < ns; b++) {
      meta[b] = B.sd_h[b].off;
      meta[ns + b] = B.probs[B.sd_h[b].prob]->ndof;
      meta[2 * ns + b] = pick[b];
    }
    long long* md = (long long*)meta_b.get(sizeof(long long) * meta.size(), B.device);
    RBWS_HIP(hipMemcpyAsync(md, meta.data(), sizeof(long long) * meta.size(), hipMemcpyHostToDevice, s));
    std::vector<int> pk(pick);
    int* pd = (int*)rows_b.get(sizeof(int) * ns, B.device);
    RBWS_HIP(hipMemcpyAsync(pd, pk.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_pick, dim3(256, ns), dim3(256), 0, s, x, (const double*)tmp, (const long long*)md,
                       (const long long*)(md + ns), (const int*)pd);
    RBWS_HIP(hipGetLastError());
    RBWS_HIP(hipStreamSynchronize(s));
  }
  for (int b = 0; b < ns; b++) used[b] = pick[b] ? RBWS_INIT_RB : RBWS_INIT_LEARNED;
}

}  // namespace rbws

using namespace rbws;

#define API_BEGIN try {
#define API_END                                              \
  }                                                          \
  catch (const Error& e) {                                   \
    set_error(e.msg);                                        \
    return e.code;                                           \
  }                                                          \
  catch (const std::bad_alloc&) {                            \
    set_error("host allocation failed");                     \
    return RBWS_ENOMEM;                                      \
  }                                                          \
  catch (const std::exception& e) {                          \
    set_error(e.what());                                     \
    return RBWS_EDEVICE;                                     \
  }                                                          \
  return RBWS_OK;

static inline Problem* PP(rbws_problem* p) { return reinterpret_cast<Problem*>(p); }
static inline const Problem* PP(const rbws_problem* p) { return reinterpret_cast<const Problem*>(p); }
static inline Basis* BB(rbws_basis* b) { return reinterpret_cast<Basis*>(b); }
static inline const Basis* BB(const rbws_basis* b) { return reinterpret_cast<const Basis*>(b); }
static inline Mlp* MM(rbws_mlp* m) { return reinterpret_cast<Mlp*>(m); }
static inline const Mlp* MM(const rbws_mlp* m) { return reinterpret_cast<const Mlp*>(m); }

extern "C" {

const char* rbws_last_error(void) { return g_err.c_str(); }
const char* rbws_version(void) { return "rbws 0.1 (gfx950)"; }

void rbws_solve_opts_default(rbws_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-10;
  o->max_iter = 50000;
  o->precond = RBWS_PREC_JACOBI;
  o->precision = RBWS_FP64;
  o->init = RBWS_INIT_ZERO;
  o->lift = RBWS_LIFT_EXACT;
  o->eta_inner = 0.1;
  o->max_outer = 40;
  o->fallback = 0;
  o->flags = 0;
  o->check_every = 0;
  o->ir_mode = RBWS_IR_RELIABLE;
  o->mg_nu = 1;
  o->mg_omega = 6.0 / 7.0;
}

rbws_status rbws_problem_create(const rbws_problem_desc* desc, int device, rbws_problem** out) {
  API_BEGIN
  RBWS_REQUIRE(out != nullptr, RBWS_EINVAL, "out is NULL");
  *out = nullptr;
  Problem* P = problem_create(desc, device);
  *out = reinterpret_cast<rbws_problem*>(P);
  API_END
}

void rbws_problem_destroy(rbws_problem* p) { problem_destroy(PP(p)); }

rbws_status rbws_problem_info(const rbws_problem* p, int* n, int* np, int* nq, long long* ndof) {
  API_BEGIN
  RBWS_REQUIRE(p != nullptr, RBWS_EINVAL, "problem is NULL");
  const Problem* P = PP(p);
  if (n) *n = P->n;
  if (np) *np = P->p;
  if (nq) *nq = P->Q;
  if (ndof) *ndof = P->ndof;
  API_END
}

rbws_status rbws_theta(const rbws_problem* p, const double* mu, int nmu, double* theta) {
  API_BEGIN
  RBWS_REQUIRE(p != nullptr, RBWS_EINVAL, "problem is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  RBWS_REQUIRE(nmu == 0 || (mu && theta), RBWS_EINVAL, "mu/theta is NULL");
  const Problem* P = PP(p);
  for (int b = 0; b < nmu; b++) theta_host(*P, mu + (long long)b * P->p, theta + (long long)b * P->Q);
  API_END
}

rbws_status rbws_spmv(rbws_problem* p, const double* mu, int nmu, const void* x, void* y,
                      int precision, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(p != nullptr, RBWS_EINVAL, "problem is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  RBWS_REQUIRE(precision == RBWS_FP64 || precision == RBWS_FP32_IR, RBWS_EINVAL, "bad precision");
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(mu && x && y, RBWS_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  static thread_local Batch& B = *new Batch();
  std::vector<const Problem*> probs{PP(p)};
  batch_setup(B, probs, nullptr, nmu, mu, PP(p)->p, s);
  spmv_batch(B, x, y, precision == RBWS_FP32_IR, s);
  RBWS_HIP(hipStreamSynchronize(s));
  API_END
}

rbws_status rbws_mg_apply(rbws_problem* p, const double* mu, int nmu, int nu, double omega, const void* r,
                          void* s, int precision, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(p != nullptr, RBWS_EINVAL, "problem is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  RBWS_REQUIRE(precision == RBWS_FP64 || precision == RBWS_FP32_IR, RBWS_EINVAL, "bad precision");
  RBWS_REQUIRE(nu >= 1 && nu <= 8 && omega > 0.0 && omega <= 1.0, RBWS_EINVAL,
               "bad multigrid settings (nu in 1..8, omega in (0, 1])");
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(mu && r && s, RBWS_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  static thread_local Batch& B = *new Batch();
  std::vector<const Problem*> probs{PP(p)};
  batch_setup(B, probs, nullptr, nmu, mu, PP(p)->p, st);
  mg_apply_all(B, nu, omega, precision == RBWS_FP32_IR, r, s, st);
  API_END
}

rbws_status rbws_exact_dots(const double* x, const double* y, long long len, int count, double* out,
                            int flags, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(len >= 0 && count >= 0, RBWS_EINVAL, "negative size");
  if (count == 0) return RBWS_OK;
  RBWS_REQUIRE(out != nullptr, RBWS_EINVAL, "out is NULL");
  if (len == 0) {
    for (int i = 0; i < count; i++) out[i] = 0.0;
    return RBWS_OK;
  }
  RBWS_REQUIRE(x && y, RBWS_EINVAL, "NULL pointer");
  exact_dots(x, y, len, count, out, flags, (hipStream_t)stream);
  API_END
}

rbws_status rbws_stream_copy(const void* src, void* dst, long long bytes, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(bytes >= 0 && bytes % 16 == 0, RBWS_EINVAL, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return RBWS_OK;
  RBWS_REQUIRE(src && dst, RBWS_EINVAL, "NULL pointer");
  RBWS_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, RBWS_EINVAL, "src and dst must be 16-byte aligned");
  stream_copy(src, dst, bytes, (hipStream_t)stream);
  API_END
}

rbws_status rbws_exact_dots_noalloc(const double* x, const double* y, long long len, int count, double* out,
                                    int flags, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(len >= 0 && count >= 0, RBWS_EINVAL, "negative size");
  if (count == 0) return RBWS_OK;
  RBWS_REQUIRE(out != nullptr, RBWS_EINVAL, "out is NULL");
  RBWS_REQUIRE(len == 0 || (x && y), RBWS_EINVAL, "NULL pointer");
  exact_dots_noalloc(x, y, len, count, out, flags, (hipStream_t)stream);
  API_END
}

rbws_status rbws_rb_build(rbws_problem* p, const double* mu_train, int ntrain, int N, double snap_tol,
                          int precond, int snap_maxit, void* stream, rbws_basis** out, int* selected,
                          double* indicator_hist, int* n_reached) {
  API_BEGIN
  RBWS_REQUIRE(p && mu_train && out, RBWS_EINVAL, "NULL argument");
  RBWS_REQUIRE(precond == RBWS_PREC_NONE || precond == RBWS_PREC_JACOBI, RBWS_EINVAL, "bad precond");
  RBWS_REQUIRE(snap_maxit >= 1, RBWS_EINVAL, "snap_maxit < 1");
  *out = nullptr;
  Basis* b = rb_build(PP(p), mu_train, ntrain, N, snap_tol, precond, snap_maxit, 0, (hipStream_t)stream);
  if (selected)
    for (int i = 0; i < N; i++) selected[i] = i < b->N ? b->selected[i] : -1;
  if (indicator_hist)
    for (size_t i = 0; i < (size_t)N * ntrain; i++)
      indicator_hist[i] = i < b->hist.size() ? b->hist[i] : std::nan("");
  if (n_reached) *n_reached = b->N;
  *out = reinterpret_cast<rbws_basis*>(b);
  API_END
}

rbws_status rbws_rb_build_l1roc(rbws_problem* p, const double* mu_train, int ntrain, int N, double snap_tol,
                                int precond, int snap_maxit, void* stream, rbws_basis** out, int* selected,
                                double* indicator_hist, int* n_reached) {
  API_BEGIN
  RBWS_REQUIRE(p && mu_train && out, RBWS_EINVAL, "NULL argument");
  RBWS_REQUIRE(precond == RBWS_PREC_NONE || precond == RBWS_PREC_JACOBI, RBWS_EINVAL, "bad precond");
  RBWS_REQUIRE(snap_maxit >= 1, RBWS_EINVAL, "snap_maxit < 1");
  *out = nullptr;
  Basis* b = rb_build_l1roc(PP(p), mu_train, ntrain, N, snap_tol, precond, snap_maxit, 0, (hipStream_t)stream);
  if (selected)
    for (int i = 0; i < N; i++) selected[i] = i < b->N ? b->selected[i] : -1;
  if (indicator_hist)
    for (size_t i = 0; i < (size_t)N * ntrain; i++)
      indicator_hist[i] = i < b->hist.size() ? b->hist[i] : std::nan("");
  if (n_reached) *n_reached = b->N;
  *out = reinterpret_cast<rbws_basis*>(b);
  API_END
}

rbws_status rbws_basis_l1roc(const rbws_basis* b, int* npts, long long* pts, int* nxs, long long* xs, int* nxr,
                             long long* xr, double* T) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  const Basis* B = BB(b);
  RBWS_REQUIRE(B->kind == 1, RBWS_ESTATE, "not an L1ROC basis");
  if (npts) *npts = (int)B->pts.size();
  if (pts) std::copy(B->pts.begin(), B->pts.end(), pts);
  if (nxs) *nxs = (int)B->xs.size();
  if (xs) std::copy(B->xs.begin(), B->xs.end(), xs);
  if (nxr) *nxr = (int)B->xr.size();
  if (xr) std::copy(B->xr.begin(), B->xr.end(), xr);
  if (T)
    for (int i = 0; i < B->N; i++)
      for (int j = 0; j < B->N; j++) T[(size_t)i * B->N + j] = B->T[(size_t)i * B->Nmax + j];
  API_END
}

void rbws_basis_destroy(rbws_basis* b) { delete BB(b); }

rbws_status rbws_basis_info(const rbws_basis* b, int* N, int* nq, long long* ndof, double* final_max) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  const Basis* B = BB(b);
  if (N) *N = B->N;
  if (nq) *nq = B->Q;
  if (ndof) *ndof = B->ndof;
  if (final_max) *final_max = B->final_max;
  API_END
}

rbws_status rbws_basis_get(const rbws_basis* b, double* V, double* AqN, double* fN) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  const Basis* B = BB(b);
  if (V) {
    RBWS_HIP(hipSetDevice(B->prob->device));
    RBWS_HIP(hipMemcpy(V, B->V.ptr, sizeof(double) * B->N * B->ndof, hipMemcpyDeviceToHost));
  }
  RBWS_REQUIRE(B->kind == 0 || (!AqN && !fN), RBWS_EINVAL, "an L1ROC basis has no reduced matrices");
  if (AqN)
    for (int q = 0; q < B->Q; q++)
      for (int i = 0; i < B->N; i++)
        for (int j = 0; j < B->N; j++)
          AqN[((size_t)q * B->N + i) * B->N + j] = B->AqN[((size_t)q * B->Nmax + i) * B->Nmax + j];
  if (fN)
    for (int i = 0; i < B->N; i++) fN[i] = B->fN[i];
  API_END
}

rbws_status rbws_basis_device_v(const rbws_basis* b, const double** V) {
  API_BEGIN
  RBWS_REQUIRE(b && V, RBWS_EINVAL, "NULL argument");
  *V = (const double*)BB(b)->V.ptr;
  API_END
}

rbws_status rbws_rb_coeffs(const rbws_basis* b, const double* mu, int nmu, double* c, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(mu && c, RBWS_EINVAL, "NULL argument");
  const Basis* B = BB(b);
  hipStream_t s = (hipStream_t)stream;
  static thread_local Batch& bt = *new Batch();
  RBWS_SCRATCH(cb);
  std::vector<const Problem*> probs{B->prob};
  batch_setup(bt, probs, nullptr, nmu, mu, B->prob->p, s);
  double* cd = (double*)cb.get(sizeof(double) * nmu * B->N, bt.device);
  std::vector<const Basis*> bl{B};
  const int bad = rb_coeffs(bt, bl, cd, B->N, 0, s);
  RBWS_REQUIRE(bad == 0, RBWS_ENUMERIC, "reduced matrix not positive definite");
  RBWS_HIP(hipMemcpyAsync(c, cd, sizeof(double) * nmu * B->N, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  API_END
}

rbws_status rbws_rb_residual_estimate(const rbws_basis* b, const double* mu, int nmu, const double* c, double* rel,
                                      void* stream) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(mu && c && rel, RBWS_EINVAL, "NULL argument");
  const Basis* B = BB(b);
  RBWS_REQUIRE(B->est, RBWS_ESTATE, "the basis has no residual decomposition");
  hipStream_t s = (hipStream_t)stream;
  static thread_local Batch& bt = *new Batch();
  RBWS_SCRATCH(cb);
  std::vector<const Problem*> probs{B->prob};
  batch_setup(bt, probs, nullptr, nmu, mu, B->prob->p, s);
  double* cd = (double*)cb.get(sizeof(double) * nmu * B->N, bt.device);
  RBWS_HIP(hipMemcpyAsync(cd, c, sizeof(double) * nmu * B->N, hipMemcpyHostToDevice, s));
  std::vector<const Basis*> bl{B};
  rb_resid_estimate(bt, bl, cd, B->N, rel, s);
  API_END
}

rbws_status rbws_rb_lift(const rbws_basis* b, const double* c, int nmu, double* u, int mode, void* stream) {
  API_BEGIN
  RBWS_REQUIRE(b != nullptr, RBWS_EINVAL, "basis is NULL");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  RBWS_REQUIRE(mode == RBWS_LIFT_EXACT || mode == RBWS_LIFT_MFMA, RBWS_EINVAL, "bad lift mode");
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(c && u, RBWS_EINVAL, "NULL argument");
  const Basis* B = BB(b);
  hipStream_t s = (hipStream_t)stream;
  static thread_local Batch& bt = *new Batch();
  std::vector<const Problem*> probs{B->prob};
  std::vector<double> th((size_t)nmu * B->Q, 1.0);
  batch_setup(bt, probs, nullptr, nmu, nullptr, B->prob->p, s, th.data());
  std::vector<const Basis*> bl{B};
  if (mode == RBWS_LIFT_EXACT) rb_lift_exact(bt, bl, c, B->N, u, 0, s);
  else rb_lift_mfma(bt, B, c, B->N, u, s);
  RBWS_HIP(hipStreamSynchronize(s));
  API_END
}

rbws_status rbws_basis_save(const rbws_basis* b, const char* path) {
  API_BEGIN
  basis_save(BB(b), path);
  API_END
}

rbws_status rbws_basis_load(rbws_problem* p, const char* path, rbws_basis** out) {
  API_BEGIN
  RBWS_REQUIRE(p && path && out, RBWS_EINVAL, "NULL argument");
  *out = nullptr;
  *out = reinterpret_cast<rbws_basis*>(basis_load(PP(p), path, nullptr));
  API_END
}

rbws_status rbws_set_tuning(int key, int value) {
  API_BEGIN
  if (key == RBWS_TUNE_SWEEP32) {
    RBWS_REQUIRE(value >= 0 && value <= 3, RBWS_EINVAL, "value out of range");
    set_sweep32_variant(value);
  } else if (key == RBWS_TUNE_GRID) {
    RBWS_REQUIRE(value == 0 || value == 1, RBWS_EINVAL, "value out of range");
    set_grid_mode(value);
  } else if (key == RBWS_TUNE_TZ) {
    RBWS_REQUIRE(value == 0 || (value >= 4 && value <= 64 && (value & (value - 1)) == 0), RBWS_EINVAL,
                 "tile depth must be 0 or a power of two in [4, 64]");
    set_tile_depth(value);
  } else if (key == RBWS_TUNE_MG_PZ) {
    RBWS_REQUIRE(value == 0 || value == 1, RBWS_EINVAL, "value out of range");
    set_mg_pz(value);
  } else {
    throw Error{RBWS_EINVAL, "unknown tuning key"};
  }
  API_END
}

rbws_status rbws_autotune(rbws_problem* p, int nsolve, int precision, void* stream, int* tz, double* ms) {
  API_BEGIN
  RBWS_REQUIRE(p != nullptr && tz != nullptr, RBWS_EINVAL, "NULL argument");
  RBWS_REQUIRE(precision == RBWS_FP64 || precision == RBWS_FP32_IR, RBWS_EINVAL, "bad precision");
  *tz = autotune_tiles(PP(p), nsolve, precision == RBWS_FP32_IR, (hipStream_t)stream, ms);
  API_END
}

rbws_status rbws_autotune_clear(void) {
  API_BEGIN
  clear_tile_table();
  API_END
}

rbws_status rbws_exact_fallbacks(long long* counts, int reset) {
  API_BEGIN
  RBWS_REQUIRE(counts != nullptr, RBWS_EINVAL, "counts is NULL");
  counts[0] = (long long)fallbacks_solver(reset != 0);
  counts[1] = (long long)fallbacks_rb(0, false);
  counts[2] = (long long)fallbacks_rb(1, false);
  counts[3] = (long long)fallbacks_rb(2, reset != 0);
  API_END
}

rbws_status rbws_profile(int enable, double* ms, long long* launches, int reset) {
  API_BEGIN
  KernelTimer& t = ktimer();
  t.flush();
  if (ms)
    for (int k = 0; k < KK_COUNT; k++) ms[k] = t.ms[k];
  if (launches)
    for (int k = 0; k < KK_COUNT; k++) launches[k] = t.count[k];
  if (reset)
    for (int k = 0; k < KK_COUNT; k++) {
      t.ms[k] = 0.0;
      t.count[k] = 0;
    }
  t.on = enable != 0;
  API_END
}

rbws_status rbws_solve(rbws_problem* const* problems, const rbws_basis* const* bases,
                       const rbws_mlp* const* mlps, int nprob, const int* problem_of,
                       const double* mu, int nmu, const rbws_solve_opts* opts, void* stream,
                       void* const* u_out, rbws_solve_stat* stats) {
  API_BEGIN
  RBWS_REQUIRE(problems != nullptr && nprob >= 1, RBWS_EINVAL, "no problems");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  RBWS_REQUIRE(opts != nullptr, RBWS_EINVAL, "opts is NULL");
  RBWS_REQUIRE(opts->tol >= 0.0 && std::isfinite(opts->tol), RBWS_EINVAL, "tol must be finite, >= 0");
  RBWS_REQUIRE(opts->max_iter >= 0, RBWS_EINVAL, "max_iter < 0");
  RBWS_REQUIRE(opts->precond == RBWS_PREC_NONE || opts->precond == RBWS_PREC_JACOBI ||
                   opts->precond == RBWS_PREC_MG,
               RBWS_EINVAL, "bad precond");
  RBWS_REQUIRE(opts->precond != RBWS_PREC_MG ||
                   (opts->mg_nu >= 1 && opts->mg_nu <= 8 && opts->mg_omega > 0.0 && opts->mg_omega <= 1.0),
               RBWS_EINVAL, "bad multigrid settings (mg_nu in 1..8, mg_omega in (0, 1])");
  RBWS_REQUIRE(opts->precision == RBWS_FP64 || opts->precision == RBWS_FP32_IR, RBWS_EINVAL,
               "bad precision");
  RBWS_REQUIRE(opts->init >= RBWS_INIT_ZERO && opts->init <= RBWS_INIT_LEARNED, RBWS_EINVAL, "bad init");
  (void)mlps;
  std::vector<const Problem*> probs(nprob);
  for (int q = 0; q < nprob; q++) {
    RBWS_REQUIRE(problems[q] != nullptr, RBWS_EINVAL, "problem is NULL");
    probs[q] = PP(problems[q]);
  }
  if (nmu == 0) return RBWS_OK;
  RBWS_REQUIRE(mu != nullptr, RBWS_EINVAL, "mu is NULL");
  RBWS_REQUIRE(opts->lift == RBWS_LIFT_EXACT || opts->lift == RBWS_LIFT_MFMA, RBWS_EINVAL, "bad lift");
  RBWS_REQUIRE(opts->fallback == 0 || opts->fallback == 1, RBWS_EINVAL, "bad fallback");
  std::vector<const Basis*> bl(nprob, nullptr);
  std::vector<Mlp*> ml(nprob, nullptr);
  if (opts->init != RBWS_INIT_ZERO) {
    RBWS_REQUIRE(bases != nullptr, RBWS_ESTATE, "RB and learned starts need a basis per problem");
    for (int q = 0; q < nprob; q++) {
      RBWS_REQUIRE(bases[q] != nullptr, RBWS_ESTATE, "RB and learned starts need a basis per problem");
      bl[q] = BB(bases[q]);
      RBWS_REQUIRE(bl[q]->prob == probs[q], RBWS_EINVAL, "basis belongs to another problem");
    }
  }
  if (opts->init == RBWS_INIT_LEARNED) {
    RBWS_REQUIRE(mlps != nullptr, RBWS_ESTATE, "learned start needs a network per problem");
    for (int q = 0; q < nprob; q++) {
      RBWS_REQUIRE(mlps[q] != nullptr, RBWS_ESTATE, "learned start needs a network per problem");
      ml[q] = const_cast<Mlp*>(MM(mlps[q]));
      RBWS_REQUIRE(ml[q]->d.p == probs[q]->p && ml[q]->d.nout == bl[q]->N, RBWS_EINVAL,
                   "network inputs/outputs do not match the problem and basis");
      RBWS_REQUIRE(ml[q]->device == probs[q]->device, RBWS_EINVAL, "network on another device");
    }
  }
  hipStream_t s = (hipStream_t)stream;
  static thread_local Batch& B = *new Batch();
  RBWS_SCRATCH(cbuf);
  batch_setup(B, probs, problem_of, nmu, mu, probs[0]->p, s);
  double* x = (double*)B.x.get(sizeof(double) * B.total, B.device);
  const int fe = (opts->flags & RBWS_FLAG_FORCE_EXACT_DOTS) ? 1 : 0;
  std::vector<int> used(nmu, opts->init);
  auto lift = [&](const double* c, double* out) {
    if (opts->lift == RBWS_LIFT_MFMA && nprob == 1) rb_lift_mfma(B, bl[0], c, 64, out, s);
    else rb_lift_exact(B, bl, c, 64, out, fe, s);
  };
  if (opts->init == RBWS_INIT_ZERO) {
    fill64(x, B.total, 0.0, s);
  } else if (opts->init == RBWS_INIT_RB) {
    double* cd = (double*)cbuf.get(sizeof(double) * 64 * nmu, B.device);
    RBWS_REQUIRE(rb_coeffs(B, bl, cd, 64, fe, s) == 0, RBWS_ENUMERIC, "reduced matrix not positive definite");
    lift(cd, x);
  } else {
    learned_start(B, bl, ml, problem_of, mu, opts->fallback, fe, !(opts->flags & RBWS_FLAG_EXPLICIT_FALLBACK), s,
                  lift, used);
  }
  RBWS_SCRATCH(tbuf);
  unsigned long long* tdev = (unsigned long long*)tbuf.get(sizeof(unsigned long long), B.device);
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, s, tdev);
  std::vector<const double*> sol(nmu);
  std::vector<IrHost> ir;
  if (opts->precision == RBWS_FP64) {
    CgOpts co{opts->tol, opts->max_iter, opts->precond, opts->flags, opts->check_every, opts->mg_nu,
              opts->mg_omega};
    cg_fp64_run(B, co, s);
    for (int b = 0; b < nmu; b++) sol[b] = x + B.sd_h[b].off;
  } else {
    RBWS_REQUIRE(opts->eta_inner > 0.0 && opts->eta_inner < 1.0, RBWS_EINVAL, "eta_inner must be in (0,1)");
    RBWS_REQUIRE(opts->max_outer >= 1, RBWS_EINVAL, "max_outer < 1");
    RBWS_REQUIRE(opts->max_iter >= 1, RBWS_EINVAL, "max_iter < 1 for refinement");
    RBWS_REQUIRE(opts->ir_mode == RBWS_IR_RESTART || opts->ir_mode == RBWS_IR_RELIABLE, RBWS_EINVAL,
                 "bad ir_mode");
    IrOpts io{opts->tol,         opts->eta_inner,  opts->precond,
              opts->max_iter,    opts->max_outer,  opts->flags,
              opts->check_every, opts->ir_mode == RBWS_IR_RELIABLE ? 1 : 0, opts->mg_nu, opts->mg_omega};
    ir_run(B, io, s, ir);
    for (int b = 0; b < nmu; b++) sol[b] = (ir[b].cur ? (const double*)B.r.ptr : x) + B.sd_h[b].off;
  }
  unsigned long long t0 = 0;
  RBWS_HIP(hipMemcpyAsync(&t0, tdev, sizeof t0, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  if (u_out) {
    for (int b = 0; b < nmu; b++)
      if (u_out[b])
        RBWS_HIP(hipMemcpyAsync(u_out[b], sol[b], sizeof(double) * B.probs[B.sd_h[b].prob]->ndof,
                                hipMemcpyDeviceToDevice, s));
  }
  if (stats) {
    if (opts->precision == RBWS_FP64) {
      collect_stats(B, t0, used, 0, stats, s);
    } else {
      const double khz = wall_clock_khz(B.device);
      for (int b = 0; b < nmu; b++) {
        rbws_solve_stat& o = stats[b];
        std::memset(&o, 0, sizeof o);
        o.iters = ir[b].iters;
        o.outer_iters = ir[b].outer;
        o.extra_spmv = ir[b].outer;
        o.status = ir[b].status;
        o.init_used = used[b];
        o.vcycles = ir[b].nvc;
        o.init_rr = ir[b].init_rr;
        o.final_rr = ir[b].rr;
        o.ff = ir[b].ff;
        o.t_done_ms = ir[b].t_done > t0 ? (double)(ir[b].t_done - t0) / khz : 0.0;
      }
    }
  }
  RBWS_HIP(hipStreamSynchronize(s));
  API_END
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned start
// ---------------------------------------------------------------------------
extern "C" {

rbws_status rbws_mlp_create(const rbws_mlp_desc* d, int device, const float* params, unsigned long long seed,
                            rbws_mlp** out) {
  API_BEGIN
  RBWS_REQUIRE(out != nullptr, RBWS_EINVAL, "out is NULL");
  *out = nullptr;
  *out = reinterpret_cast<rbws_mlp*>(mlp_create(d, device, params, seed));
  API_END
}

void rbws_mlp_destroy(rbws_mlp* m) { mlp_destroy(MM(m)); }

rbws_status rbws_mlp_param_count(const rbws_mlp* m, long long* count) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr && count != nullptr, RBWS_EINVAL, "NULL argument");
  *count = MM(m)->np;
  API_END
}

rbws_status rbws_mlp_info(const rbws_mlp* m, rbws_mlp_desc* d) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr && d != nullptr, RBWS_EINVAL, "NULL argument");
  *d = MM(m)->d;
  API_END
}

rbws_status rbws_mlp_get_params(const rbws_mlp* m, float* params) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  RBWS_HIP(hipSetDevice(MM(m)->device));
  mlp_get_params(MM(m), params, nullptr);
  API_END
}

rbws_status rbws_mlp_set_params(rbws_mlp* m, const float* params) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  RBWS_HIP(hipSetDevice(MM(m)->device));
  mlp_set_params(MM(m), params, nullptr);
  API_END
}

rbws_status rbws_mlp_set_output_scaling(rbws_mlp* m, const double* mean, const double* stdev) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  RBWS_HIP(hipSetDevice(MM(m)->device));
  mlp_set_scaling(MM(m), mean, stdev, nullptr);
  API_END
}

rbws_status rbws_mlp_get_output_scaling(const rbws_mlp* m, double* mean, double* stdev) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  for (int j = 0; j < MM(m)->d.nout; j++) {
    if (mean) mean[j] = MM(m)->out_mean[j];
    if (stdev) stdev[j] = MM(m)->out_std[j];
  }
  API_END
}

rbws_status rbws_mlp_fit_output_scaling(rbws_mlp* m, const double* mu, const double* c, int npairs) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  mlp_fit_scaling(MM(m), mu, c, npairs, nullptr);
  API_END
}

rbws_status rbws_mlp_predict(const rbws_mlp* m, const double* mu, int nmu, double* c) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr && c != nullptr, RBWS_EINVAL, "NULL argument");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  if (nmu == 0) return RBWS_OK;
  Mlp* mm = const_cast<Mlp*>(MM(m));
  RBWS_HIP(hipSetDevice(mm->device));
  RBWS_SCRATCH(cb);
  const int no = mm->d.nout;
  double* cd = (double*)cb.get(sizeof(double) * (size_t)nmu * no, mm->device);
  mlp_predict_dev(mm, mu, nmu, nullptr, cd, no, nullptr);
  RBWS_HIP(hipMemcpy(c, cd, sizeof(double) * (size_t)nmu * no, hipMemcpyDeviceToHost));
  API_END
}

rbws_status rbws_mlp_forward(const rbws_mlp* m, const double* mu, int nmu, float* y) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr && y != nullptr, RBWS_EINVAL, "NULL argument");
  RBWS_REQUIRE(nmu >= 0, RBWS_EINVAL, "nmu < 0");
  if (nmu == 0) return RBWS_OK;
  Mlp* mm = const_cast<Mlp*>(MM(m));
  RBWS_HIP(hipSetDevice(mm->device));
  const float* o = mlp_forward_host(mm, mu, nmu, nullptr);
  const int ld = mm->outp[mm->L - 1], no = mm->d.nout;
  std::vector<float> h((size_t)nmu * ld);
  RBWS_HIP(hipMemcpy(h.data(), o, sizeof(float) * h.size(), hipMemcpyDeviceToHost));
  for (int r = 0; r < nmu; r++)
    for (int j = 0; j < no; j++) y[(size_t)r * no + j] = h[(size_t)r * ld + j];
  API_END
}

rbws_status rbws_mlp_grad(rbws_mlp* m, const double* mu, const double* c, int nb, double* loss, float* grads) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  const double l = mlp_grad(MM(m), mu, c, nb, grads, nullptr);
  if (loss) *loss = l;
  API_END
}

rbws_status rbws_mlp_adam_step(rbws_mlp* m, const double* mu, const double* c, int nb, double lr, double* loss) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  const double l = mlp_adam_step(MM(m), mu, c, nb, lr, nullptr);
  if (loss) *loss = l;
  API_END
}

rbws_status rbws_mlp_train(rbws_mlp* m, const double* mu, const double* c, int npairs,
                           const rbws_mlp_train_cfg* cfg, double* loss_hist) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  RBWS_REQUIRE(npairs >= 1, RBWS_EINVAL, "npairs < 1");
  mlp_train(MM(m), mu, c, npairs, cfg, loss_hist, nullptr);
  API_END
}

rbws_status rbws_mlp_save(const rbws_mlp* m, const char* path) {
  API_BEGIN
  RBWS_REQUIRE(m != nullptr, RBWS_EINVAL, "network is NULL");
  RBWS_HIP(hipSetDevice(MM(m)->device));
  mlp_save(MM(m), path);
  API_END
}

rbws_status rbws_mlp_load(const char* path, int device, rbws_mlp** out) {
  API_BEGIN
  RBWS_REQUIRE(out != nullptr, RBWS_EINVAL, "out is NULL");
  *out = nullptr;
  *out = reinterpret_cast<rbws_mlp*>(mlp_load(path, device));
  API_END
}

}  // extern "C"
