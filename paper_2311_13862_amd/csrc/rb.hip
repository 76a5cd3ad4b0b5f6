// rb.hip -- reduced basis on gfx950.
//
// Offline (the paper's Alg. 4 skeleton with a residual-norm indicator):
//   snapshot u(mu_l) by the batched PCG from zero; two classical Gram-Schmidt
//   passes against V (each coefficient and each updated entry one correctly
//   rounded dot); v_n = v / ||v||; W_q = A_q v_n for every affine term (the
//   stencil with theta = e_q); A_q^N[i][n] = A_q^N[n][i] = v_i . W_q and
//   f^N[n] = v_n . f; then the indicator ||f - A(mu) V c(mu)|| / ||f|| for the
//   whole training set, evaluated directly (lift, stencil, norm); the next
//   parameter is the first maximiser.
// Online (Eq. "RB system"): A_N(mu) = sum_q theta_q A_q^N (fma in q order),
//   Cholesky and two triangular solves in one wavefront per parameter, every
//   inner sum a correctly rounded dot; then the lift u0 = V c.
// Two lifts: exact (each entry a correctly rounded N-term dot; used where the
// FP64 trajectory must be reproducible) and FP64 MFMA (v_mfma_f64_16x16x4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "rb.hpp"
#include "stencil.hpp"

namespace rbws {

constexpr int kMaxN = 64;
constexpr int kRedoCap = 1 << 20;

// exact-path fallbacks of this translation unit: [0] pair dots, [1] per-entry
// redo (Gram-Schmidt, lift), [2] reduced Cholesky and triangular solves
__device__ unsigned long long g_fallback_rb[3];

unsigned long long fallbacks_rb(int which, bool reset) {
  unsigned long long v[3] = {0, 0, 0};
  RBWS_HIP(hipMemcpyFromSymbol(v, HIP_SYMBOL(g_fallback_rb), sizeof v));
  if (reset) {
    const unsigned long long z[3] = {0, 0, 0};
    RBWS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_fallback_rb), z, sizeof z));
  }
  return v[which];
}

// ---------------------------------------------------------------------------
// dots of pointer pairs: out[v] = xs[v] . ys[v], all of length len
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pdot_part(const double* const* xs, const double* const* ys,
                                                   long long len, int per_block, CrAcc* part) {
  __shared__ CrAcc red[4];
  const int v = blockIdx.y;
  const double* X = xs[v];
  const double* Y = ys[v];
  const long long beg = (long long)blockIdx.x * per_block, end = min(len, beg + per_block);
  CrAcc a = cr_zero();
  for (long long c = beg + threadIdx.x; c < end; c += blockDim.x) cr_add_prod(a, X[c], Y[c]);
  a = cr_block_reduce(a, red);
  if (threadIdx.x == 0) part[(long long)v * gridDim.x + blockIdx.x] = a;
}

struct DotShared {
  CrAcc red[4];
  XAcc xa;
  uint32_t dig[XA_WORDS];
  double val;
  int ok;
};

__global__ __launch_bounds__(256) void k_pdot_fin(const double* const* xs, const double* const* ys,
                                                  long long len, int nparts, const CrAcc* part,
                                                  double* out, int force_exact) {
  __shared__ DotShared sh;
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
  if (threadIdx.x == 0) atomicAdd(&g_fallback_rb[0], 1ull);
  __syncthreads();
  xa_clear(&sh.xa);
  __syncthreads();
  const double* X = xs[v];
  const double* Y = ys[v];
  for (long long c = threadIdx.x; c < len; c += blockDim.x) xa_add_prod(&sh.xa, X[c], Y[c]);
  __syncthreads();
  if (threadIdx.x == 0) out[v] = xa_round(&sh.xa, sh.dig);
}

// out (device) = correctly rounded dots of the pairs (host pointer lists)
static void pair_dots(const std::vector<const double*>& xs, const std::vector<const double*>& ys,
                      long long len, double* out_dev, int force_exact, int dev, hipStream_t s) {
  const int count = (int)xs.size();
  if (count == 0) return;
  RBWS_SCRATCH(ptrs);
  RBWS_SCRATCH(part);
  const int per_block = 8192;
  const long long nb = std::max<long long>(1, (len + per_block - 1) / per_block);
  const double** pp = (const double**)ptrs.get(sizeof(double*) * 2 * count, dev);
  std::vector<const double*> h(xs);
  h.insert(h.end(), ys.begin(), ys.end());
  RBWS_HIP(hipMemcpyAsync(pp, h.data(), sizeof(double*) * 2 * count, hipMemcpyHostToDevice, s));
  CrAcc* pa = (CrAcc*)part.get(sizeof(CrAcc) * nb * count, dev);
  hipLaunchKernelGGL(k_pdot_part, dim3((unsigned)nb, count), dim3(256), 0, s, pp, pp + count, len, per_block, pa);
  hipLaunchKernelGGL(k_pdot_fin, dim3(count), dim3(256), 0, s, pp, pp + count, len, (int)nb, pa, out_dev,
                     force_exact);
  RBWS_HIP(hipGetLastError());
  // the host vector `h` must outlive the asynchronous copy
  RBWS_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Gram-Schmidt update v_c = v_c - sum_j coef_j V_j,c (one correctly rounded dot per entry)
// ---------------------------------------------------------------------------
struct Redo {
  int count;
  int overflow;
  long long idx[1];  // kRedoCap entries follow
};

__device__ __forceinline__ void redo_push(Redo* r, long long e, long long cap = kRedoCap) {
  atomicAdd(&g_fallback_rb[1], 1ull);
  int slot = atomicAdd(&r->count, 1);
  if (slot < cap) r->idx[slot] = e;
  else r->overflow = 1;
}

// v <- v - sum_j coef_j V_j, each entry correctly rounded.  `redo` holds
// `cap` >= ndof entries, so it cannot overflow: the exact pass then reads the
// original v of every entry it recomputes.
__global__ __launch_bounds__(256) void k_gs_update(double* v, const double* V, const double* coef, int nb,
                                                   long long ndof, Redo* redo, int force_exact, long long cap) {
  __shared__ double cs[kMaxN];
  for (int j = threadIdx.x; j < nb; j += blockDim.x) cs[j] = -coef[j];
  __syncthreads();
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ndof;
       c += (long long)gridDim.x * blockDim.x) {
    CrAcc a = cr_zero();
    cr_add(a, v[c]);
    for (int j = 0; j < nb; j++) cr_add_prod(a, cs[j], V[(long long)j * ndof + c]);
    double r;
    if (!force_exact && cr_finalize(a, &r)) v[c] = r;
    else redo_push(redo, c, cap);
  }
}

// exact recomputation of the listed entries (one 64-thread block per entry)
__global__ __launch_bounds__(64) void k_gs_redo(double* v, const double* V, const double* coef, int nb,
                                                long long ndof, const Redo* redo) {
  __shared__ XAcc xa;
  __shared__ uint32_t dig[XA_WORDS];
  const long long total = redo->overflow ? ndof : (long long)redo->count;
  for (long long e = blockIdx.x; e < total; e += gridDim.x) {
    const long long c = redo->overflow ? e : redo->idx[e];
    __syncthreads();
    xa_clear(&xa);
    __syncthreads();
    if (threadIdx.x == 0) xa_add(&xa, v[c]);
    for (int j = threadIdx.x; j < nb; j += blockDim.x) xa_add_prod(&xa, -coef[j], V[(long long)j * ndof + c]);
    __syncthreads();
    const double r = threadIdx.x == 0 ? xa_round(&xa, dig) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) v[c] = r;
  }
}

__global__ void k_div(double* out, const double* v, const double* nrm, long long ndof) {
  const double d = *nrm;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ndof;
       c += (long long)gridDim.x * blockDim.x)
    out[c] = v[c] / d;
}

__global__ void k_copy_rep(double* dst, const double* src, long long ndof, int reps) {
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ndof * reps;
       c += (long long)gridDim.x * blockDim.x)
    dst[c] = src[c % ndof];
}

// ---------------------------------------------------------------------------
// online solve: one wavefront per parameter
// ---------------------------------------------------------------------------
struct CholShared {
  double A[kMaxN * kMaxN];  // assembled matrix; its lower triangle becomes L
  double y[kMaxN];
  double c[kMaxN];
  XAcc xa;
  uint32_t dig[XA_WORDS];
  double val;
  int ok;
};

// value of sum over lanes of the terms each lane added to `a` (all 64 lanes
// call); exact fallback adds the same terms through `add_terms`
template <typename S, typename F>
__device__ __forceinline__ double wave_sum(S& sh, CrAcc a, int force_exact, F add_terms) {
  a = cr_wave_reduce(a);
  if (threadIdx.x == 0) {
    double r = 0.0;
    sh.ok = (!force_exact && cr_finalize(a, &r)) ? 1 : 0;
    sh.val = r;
  }
  __syncthreads();
  if (!sh.ok) {
    if (threadIdx.x == 0) atomicAdd(&g_fallback_rb[2], 1ull);
    __syncthreads();
    xa_clear(&sh.xa);
    __syncthreads();
    add_terms(&sh.xa);
    __syncthreads();
    if (threadIdx.x == 0) sh.val = xa_round(&sh.xa, sh.dig);
  }
  __syncthreads();
  const double v = sh.val;
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(64) void k_rb_coeffs(const RbDev* __restrict__ rbd, const int* __restrict__ solve_of,
                                                  const double* __restrict__ theta, double* __restrict__ cout,
                                                  int cstride, int* bad, int force_exact) {
  __shared__ CholShared sh;
  const int b = solve_of ? solve_of[blockIdx.x] : (int)blockIdx.x;
  const RbDev R = rbd[b];
  const int N = R.N, ld = R.ld, lane = threadIdx.x;
  const double* th = theta + (long long)b * kMaxQ;
  for (int e = lane; e < N * N; e += 64) {
    const int i = e / N, j = e % N;
    double a = 0.0;
    for (int q = 0; q < R.Q; q++) a = __fma_rn(th[q], R.AqN[((long long)q * ld + i) * ld + j], a);
    sh.A[i * kMaxN + j] = a;
  }
  __syncthreads();
  double* A = sh.A;
  int fail = 0;
  for (int j = 0; j < N && !fail; j++) {
    // pivot: A_jj - sum_{k<j} L_jk^2
    CrAcc a = cr_zero();
    if (lane < j) cr_add_prod(a, -A[j * kMaxN + lane], A[j * kMaxN + lane]);
    if (lane == j) cr_add(a, A[j * kMaxN + j]);
    const double piv = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane < j) xa_add_prod(x, -A[j * kMaxN + lane], A[j * kMaxN + lane]);
      if (lane == j) xa_add(x, A[j * kMaxN + j]);
    });
    if (!(piv > 0.0) || !__builtin_isfinite(piv)) { fail = 1; break; }
    const double ljj = sqrt(piv);
    // column j below the diagonal: lane i computes its own entry
    double lij = 0.0;
    int amb = 0;
    if (lane > j && lane < N) {
      CrAcc t = cr_zero();
      cr_add(t, A[lane * kMaxN + j]);
      for (int k = 0; k < j; k++) cr_add_prod(t, -A[lane * kMaxN + k], A[j * kMaxN + k]);
      double v;
      if (!force_exact && cr_finalize(t, &v)) lij = v / ljj;
      else amb = 1;
    }
    unsigned long long m = __ballot(amb);
    while (m) {  // exact path for the rare ambiguous entries, one at a time
      const int i = __ffsll((long long)m) - 1;
      if (lane == 0) atomicAdd(&g_fallback_rb[2], 1ull);
      m &= m - 1;
      __syncthreads();
      xa_clear(&sh.xa);
      __syncthreads();
      if (lane == 0) xa_add(&sh.xa, A[i * kMaxN + j]);
      if (lane < j) xa_add_prod(&sh.xa, -A[i * kMaxN + lane], A[j * kMaxN + lane]);
      __syncthreads();
      if (lane == 0) sh.val = xa_round(&sh.xa, sh.dig);
      __syncthreads();
      if (lane == i) lij = sh.val / ljj;
    }
    __syncthreads();
    if (lane > j && lane < N) A[lane * kMaxN + j] = lij;
    if (lane == j) A[j * kMaxN + j] = ljj;
    __syncthreads();
  }
  if (fail) {
    if (lane == 0) atomicAdd(bad, 1);
    for (int i = lane; i < N; i += 64) cout[(long long)b * cstride + i] = __builtin_nan("");
    return;
  }
  // forward: L y = b_N
  for (int i = 0; i < N; i++) {
    CrAcc a = cr_zero();
    if (lane < i) cr_add_prod(a, -A[i * kMaxN + lane], sh.y[lane]);
    if (lane == i) cr_add(a, R.fN[i]);
    const double v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane < i) xa_add_prod(x, -A[i * kMaxN + lane], sh.y[lane]);
      if (lane == i) xa_add(x, R.fN[i]);
    });
    if (lane == 0) sh.y[i] = v / A[i * kMaxN + i];
    __syncthreads();
  }
  // back: L^T c = y
  for (int i = N - 1; i >= 0; i--) {
    CrAcc a = cr_zero();
    if (lane > i && lane < N) cr_add_prod(a, -A[lane * kMaxN + i], sh.c[lane]);
    if (lane == i) cr_add(a, sh.y[i]);
    const double v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane > i && lane < N) xa_add_prod(x, -A[lane * kMaxN + i], sh.c[lane]);
      if (lane == i) xa_add(x, sh.y[i]);
    });
    if (lane == 0) sh.c[i] = v / A[i * kMaxN + i];
    __syncthreads();
  }
  for (int i = lane; i < N; i += 64) cout[(long long)b * cstride + i] = sh.c[i];
}

// ---------------------------------------------------------------------------
// exact lift: u[b][c] = sum_j V[j][c] C[b][j], each a correctly rounded dot.
// A block owns 64 points; their V values stay in LDS while it walks solves.
// ---------------------------------------------------------------------------
constexpr int kLiftPts = 64;
constexpr int kLiftGroup = 32;  // solves per block

__global__ __launch_bounds__(256) void k_lift_exact(const double* __restrict__ V, int N, long long ndof,
                                                    const int* __restrict__ solves, int nsol,
                                                    const long long* __restrict__ off,
                                                    const double* __restrict__ C, int cstride,
                                                    double* __restrict__ u, Redo* redo, int force_exact) {
  __shared__ double vt[kMaxN * kLiftPts];
  const long long c0 = (long long)blockIdx.x * kLiftPts;
  const int pl = threadIdx.x % kLiftPts, sl = threadIdx.x / kLiftPts;
  for (int e = threadIdx.x; e < N * kLiftPts; e += blockDim.x) {
    const int j = e / kLiftPts, q = e % kLiftPts;
    vt[e] = (c0 + q < ndof) ? V[(long long)j * ndof + c0 + q] : 0.0;
  }
  __syncthreads();
  const long long c = c0 + pl;
  if (c >= ndof) return;
  const int g0 = blockIdx.y * kLiftGroup;
  for (int t = g0 + sl; t < min(nsol, g0 + kLiftGroup); t += blockDim.x / kLiftPts) {
    const int b = solves ? solves[t] : t;
    const double* cb = C + (long long)b * cstride;
    CrAcc a = cr_zero();
    for (int j = 0; j < N; j++) cr_add_prod(a, vt[j * kLiftPts + pl], cb[j]);
    double r;
    const long long e = off[b] + c;
    if (!force_exact && cr_finalize(a, &r)) u[e] = r;
    else redo_push(redo, ((long long)t << 32) | c);
  }
}

__global__ __launch_bounds__(64) void k_lift_redo(const double* V, int N, long long ndof, const int* solves,
                                                  int nsol, const long long* off, const double* C,
                                                  int cstride, double* u, const Redo* redo) {
  __shared__ XAcc xa;
  __shared__ uint32_t dig[XA_WORDS];
  const long long total = redo->overflow ? ndof * nsol : (long long)redo->count;
  for (long long e = blockIdx.x; e < total; e += gridDim.x) {
    long long t, c;
    if (redo->overflow) { t = e / ndof; c = e % ndof; }
    else { t = redo->idx[e] >> 32; c = redo->idx[e] & 0xffffffffll; }
    const int b = solves ? solves[t] : (int)t;
    const double* cb = C + (long long)b * cstride;
    __syncthreads();
    xa_clear(&xa);
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) xa_add_prod(&xa, V[(long long)j * ndof + c], cb[j]);
    __syncthreads();
    const double r = threadIdx.x == 0 ? xa_round(&xa, dig) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) u[off[b] + c] = r;
  }
}

// ---------------------------------------------------------------------------
// MFMA lift: U (solves x points) = C (solves x N) * V (N x points), FP64
// v_mfma_f64_16x16x4: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i % 4), register i / 4.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_lift_mfma(const double* __restrict__ V, int N, long long ndof,
                                                   const int* __restrict__ solves, int nsol,
                                                   const long long* __restrict__ off,
                                                   const double* __restrict__ C, int cstride,
                                                   double* __restrict__ u) {
  // a wave owns two 16-point column tiles (two independent MFMA chains sharing
  // the C fragments); the C fragments of the next 16 solves are loaded while
  // the current ones are multiplied
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long c0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (c0 >= ndof) return;
  const int col = lane & 15, kq = lane >> 4;
  const long long cc0 = c0 + col, cc1 = c0 + 16 + col;
  const bool in0 = cc0 < ndof, in1 = cc1 < ndof;
  // V fragments of the two tiles: K = N padded to a multiple of 4
  double v0[kMaxN / 4], v1[kMaxN / 4];
  const int ksteps = (N + 3) / 4;
#pragma unroll
  for (int s = 0; s < kMaxN / 4; s++) {
    const int k = 4 * s + kq;
    const bool kin = s < ksteps && k < N;
    v0[s] = (kin && in0) ? V[(long long)k * ndof + cc0] : 0.0;
    v1[s] = (kin && in1) ? V[(long long)k * ndof + cc1] : 0.0;
  }
  auto load_a = [&](int t0, double a[kMaxN / 4]) __attribute__((always_inline)) {
    const int ta = t0 + col;  // the solve row this lane feeds into A
    const int ba = ta < nsol ? (solves ? solves[ta] : ta) : -1;
#pragma unroll
    for (int s = 0; s < kMaxN / 4; s++) {
      const int k = 4 * s + kq;
      a[s] = (s < ksteps && ba >= 0 && k < N) ? C[(long long)ba * cstride + k] : 0.0;
    }
  };
  double a[kMaxN / 4], an[kMaxN / 4];
  load_a(0, a);
  for (int t0 = 0; t0 < nsol; t0 += 16) {
    if (t0 + 16 < nsol) load_a(t0 + 16, an);
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kMaxN / 4; s++) {
      if (s < ksteps) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], v0[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], v1[s], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int t = t0 + 4 * r + kq;
      if (t < nsol) {
        const int b = solves ? solves[t] : t;
        if (in0) u[off[b] + cc0] = acc0[r];
        if (in1) u[off[b] + cc1] = acc1[r];
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxN / 4; s++) a[s] = an[s];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void Basis::upload(hipStream_t s) {
  const int dev = prob->device;
  if (kind == 1) {
    long long* pd = (long long*)pts_d.get(sizeof(long long) * std::max<size_t>(pts.size(), 1), dev);
    RBWS_HIP(hipMemcpyAsync(pd, pts.data(), sizeof(long long) * pts.size(), hipMemcpyHostToDevice, s));
    double* td = (double*)T_d.get(sizeof(double) * T.size(), dev);
    RBWS_HIP(hipMemcpyAsync(td, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, s));
  }
  if (est) {
    double* gd = (double*)G_d.get(sizeof(double) * G.size(), dev);
    RBWS_HIP(hipMemcpyAsync(gd, G.data(), sizeof(double) * G.size(), hipMemcpyHostToDevice, s));
    double* gv = (double*)g_d.get(sizeof(double) * g.size(), dev);
    RBWS_HIP(hipMemcpyAsync(gv, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, s));
  }
  double* a = (double*)AqN_d.get(sizeof(double) * AqN.size(), dev);
  RBWS_HIP(hipMemcpyAsync(a, AqN.data(), sizeof(double) * AqN.size(), hipMemcpyHostToDevice, s));
  double* f = (double*)fN_d.get(sizeof(double) * fN.size(), dev);
  RBWS_HIP(hipMemcpyAsync(f, fN.data(), sizeof(double) * fN.size(), hipMemcpyHostToDevice, s));
  RBWS_HIP(hipStreamSynchronize(s));
}

static RbDev rbdev_of(const Basis* bs) {
  RbDev r;
  r.AqN = (const double*)bs->AqN_d.ptr;
  r.fN = (const double*)bs->fN_d.ptr;
  r.V = (const double*)bs->V.ptr;
  r.N = bs->N;
  r.ld = bs->Nmax;
  r.Q = bs->Q;
  r.pad = 0;
  return r;
}

// ---------------------------------------------------------------------------
// reduced right-hand side of a parameter-dependent source: b_N(mu) = V^T f(mu)
// (the Gaussian source is not affine in mu, so it is projected per solve).
// An FP64 matrix-core contraction over the points, with f generated in
// registers: a workgroup takes a chunk of points and 16 solves, each wave 16
// basis vectors; per step of 4 points, lane (i + 16 k) feeds V[j0 + i][c + k]
// and f_{s0 + i}(c + k).  Chunks are summed in order by a second kernel, so
// the result is deterministic (but not correctly rounded).
// ---------------------------------------------------------------------------
constexpr int kProjChunk = 4096;

__global__ __launch_bounds__(256) void k_project(const double* __restrict__ V, int N, long long ndof,
                                                 const ProbDev* __restrict__ pd, const SolveDev* __restrict__ sd,
                                                 const int* __restrict__ solves, int nsol,
                                                 double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = wave * 16;
  if (j0 >= N) return;
  const int col = lane & 15, kq = lane >> 4;
  const int s0 = blockIdx.y * 16;
  const int sb = s0 + col < nsol ? solves[s0 + col] : -1;
  const long long c0 = (long long)blockIdx.x * kProjChunk, c1 = min(ndof, c0 + kProjChunk);
  const ProbDev& P = *pd;
  const int n = P.g.n;
  SolveDev S{};
  if (sb >= 0) S = sd[sb];
  const bool arow = j0 + col < N;
  const double* vr = V + (long long)(arow ? j0 + col : 0) * ndof;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (long long c = c0; c < c1; c += 4) {
    const long long cc = c + kq;
    const bool in = cc < c1;
    const double a = (arow && in) ? vr[cc] : 0.0;
    double b = 0.0;
    if (sb >= 0 && in) {
      const int i = (int)(cc % n) + 1, j = (int)((cc / n) % n) + 1, k = (int)(cc / ((long long)n * n)) + 1;
      b = fval_fast(P, S, i, j, k);
    }
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // acc[r] = sum over the chunk of V[j0 + kq + 4 r][c] f_{s0 + col}(c)
  if (s0 + col < nsol) {
    double* out = part + ((long long)blockIdx.x * nsol + s0 + col) * kMaxN;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int j = j0 + kq + 4 * r;
      if (j < N) out[j] = acc[r];
    }
  }
}

__global__ void k_project_fin(const double* __restrict__ part, int nchunk, int nsol, int N,
                              const int* __restrict__ solves, double* __restrict__ bN) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nsol * N) return;
  const int t = e / N, j = e % N;
  double sum = 0.0;
  for (int q = 0; q < nchunk; q++) sum += part[((long long)q * nsol + t) * kMaxN + j];
  bN[(long long)solves[t] * kMaxN + j] = sum;
}

// b_N of every solve whose problem has a parameter-dependent source, into
// bN (nsolve x kMaxN); returns false when no solve needs it
static bool project_sources(Batch& B, const std::vector<const Basis*>& bases, double* bN, hipStream_t s) {
  bool any = false;
  RBWS_SCRATCH(partb);
  RBWS_SCRATCH(solb);
  for (int q = 0; q < B.nprob; q++) {
    if (B.probs[q]->desc.f_kind == RBWS_F_ONE) continue;
    std::vector<int> sol;
    for (int b = 0; b < B.nsolve; b++)
      if (B.sd_h[b].prob == q) sol.push_back(b);
    if (sol.empty()) continue;
    any = true;
    const Basis* bs = bases[q];
    const long long nd = bs->ndof;
    const int nchunk = (int)((nd + kProjChunk - 1) / kProjChunk), ns = (int)sol.size();
    double* part = (double*)partb.get(sizeof(double) * (size_t)nchunk * ns * kMaxN, B.device);
    int* sd = (int*)solb.get(sizeof(int) * ns, B.device);
    RBWS_HIP(hipMemcpyAsync(sd, sol.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_project, dim3(nchunk, (ns + 15) / 16), dim3(256), 0, s, (const double*)bs->V.ptr, bs->N,
                       nd, (const ProbDev*)B.pd.ptr + q, (const SolveDev*)B.sd.ptr, (const int*)sd, ns, part);
    hipLaunchKernelGGL(k_project_fin, dim3((ns * bs->N + 255) / 256), dim3(256), 0, s, (const double*)part, nchunk,
                       ns, bs->N, (const int*)sd, bN);
    RBWS_HIP(hipGetLastError());
    RBWS_HIP(hipStreamSynchronize(s));  // partb / solb are reused by the next problem
  }
  return any;
}

static int l1roc_coeffs(Batch& B, const std::vector<const Basis*>& bases, double* c, int cstride,
                        double* delta, int force_exact, hipStream_t s);

int rb_coeffs(Batch& B, const std::vector<const Basis*>& bases, double* c, int cstride, int force_exact,
              hipStream_t s) {
  const int ns = B.nsolve;
  if (ns == 0) return 0;
  int nl1 = 0;
  for (int b = 0; b < ns; b++) {
    const Basis* bs = bases[B.sd_h[b].prob];
    nl1 += bs != nullptr && bs->kind == 1;
  }
  if (nl1 > 0) {
    RBWS_REQUIRE(nl1 == ns, RBWS_EINVAL, "L1ROC and Galerkin bases cannot share a batch");
    return l1roc_coeffs(B, bases, c, cstride, nullptr, force_exact, s);
  }
  std::vector<RbDev> h(ns);
  for (int b = 0; b < ns; b++) {
    const Basis* bs = bases[B.sd_h[b].prob];
    RBWS_REQUIRE(bs != nullptr, RBWS_ESTATE, "a reduced basis is required for this start");
    RBWS_REQUIRE(bs->prob == B.probs[B.sd_h[b].prob], RBWS_EINVAL, "basis belongs to another problem");
    RBWS_REQUIRE(bs->N <= cstride, RBWS_EINVAL, "coefficient stride too small");
    h[b] = rbdev_of(bs);
  }
  RBWS_SCRATCH(bnb);
  double* bN = (double*)bnb.get(sizeof(double) * (size_t)ns * kMaxN, B.device);
  ktimer().begin(s, KK_PROJ);
  const bool projected = project_sources(B, bases, bN, s);
  ktimer().end(s);
  if (projected)
    for (int b = 0; b < ns; b++)
      if (B.probs[B.sd_h[b].prob]->desc.f_kind != RBWS_F_ONE) h[b].fN = bN + (size_t)b * kMaxN;
  RBWS_SCRATCH(rbd);
  RBWS_SCRATCH(badb);
  RbDev* d = (RbDev*)rbd.get(sizeof(RbDev) * ns, B.device);
  int* bad = (int*)badb.get(sizeof(int), B.device);
  RBWS_HIP(hipMemcpyAsync(d, h.data(), sizeof(RbDev) * ns, hipMemcpyHostToDevice, s));
  RBWS_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  ktimer().begin(s, KK_COEF);
  hipLaunchKernelGGL(k_rb_coeffs, dim3(ns), dim3(64), 0, s, d, (const int*)nullptr,
                     (const double*)B.theta.ptr, c, cstride, bad, force_exact);
  ktimer().end(s);
  RBWS_HIP(hipGetLastError());
  int hb = 0;
  RBWS_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  return hb;
}

// solves of batch B that belong to problem q, and the vector offsets of all solves
static void group_of(Batch& B, int q, std::vector<int>& sol) {
  sol.clear();
  for (int b = 0; b < B.nsolve; b++)
    if (B.sd_h[b].prob == q) sol.push_back(b);
}

static long long* offsets_dev(Batch& B, hipStream_t s) {
  RBWS_SCRATCH(offb);
  std::vector<long long> o(std::max(B.nsolve, 1));
  for (int b = 0; b < B.nsolve; b++) o[b] = B.sd_h[b].off;
  long long* d = (long long*)offb.get(sizeof(long long) * o.size(), B.device);
  RBWS_HIP(hipMemcpyAsync(d, o.data(), sizeof(long long) * o.size(), hipMemcpyHostToDevice, s));
  RBWS_HIP(hipStreamSynchronize(s));
  return d;
}

void rb_lift_exact(Batch& B, const std::vector<const Basis*>& bases, const double* c, int cstride,
                   double* u, int force_exact, hipStream_t s) {
  if (B.nsolve == 0) return;
  long long* off = offsets_dev(B, s);
  RBWS_SCRATCH(solb);
  RBWS_SCRATCH(redob);
  Redo* redo = (Redo*)redob.get(sizeof(Redo) + sizeof(long long) * kRedoCap, B.device);
  std::vector<int> sol;
  for (int q = 0; q < B.nprob; q++) {
    group_of(B, q, sol);
    if (sol.empty()) continue;
    const Basis* bs = bases[q];
    RBWS_REQUIRE(bs != nullptr && bs->N >= 1, RBWS_ESTATE, "a reduced basis is required for this start");
    int* sd = (int*)solb.get(sizeof(int) * sol.size(), B.device);
    RBWS_HIP(hipMemcpyAsync(sd, sol.data(), sizeof(int) * sol.size(), hipMemcpyHostToDevice, s));
    RBWS_HIP(hipMemsetAsync(redo, 0, sizeof(Redo), s));
    const long long nd = bs->ndof;
    dim3 grid((unsigned)((nd + kLiftPts - 1) / kLiftPts), (unsigned)((sol.size() + kLiftGroup - 1) / kLiftGroup));
    hipLaunchKernelGGL(k_lift_exact, grid, dim3(256), 0, s, (const double*)bs->V.ptr, bs->N, nd, sd,
                       (int)sol.size(), off, c, cstride, u, redo, force_exact);
    hipLaunchKernelGGL(k_lift_redo, dim3(1024), dim3(64), 0, s, (const double*)bs->V.ptr, bs->N, nd, sd,
                       (int)sol.size(), off, c, cstride, u, redo);
    RBWS_HIP(hipGetLastError());
    RBWS_HIP(hipStreamSynchronize(s));  // `sol` is reused by the next group
  }
}

void rb_lift_mfma(Batch& B, const Basis* bs, const double* c, int cstride, double* u, hipStream_t s) {
  if (B.nsolve == 0) return;
  RBWS_REQUIRE(bs != nullptr && bs->N >= 1, RBWS_ESTATE, "a reduced basis is required for this start");
  long long* off = offsets_dev(B, s);
  const long long nd = bs->ndof;
  const unsigned grid = (unsigned)((nd + 127) / 128);
  ktimer().begin(s, KK_LIFT);
  hipLaunchKernelGGL(k_lift_mfma, dim3(grid), dim3(256), 0, s, (const double*)bs->V.ptr, bs->N, nd,
                     (const int*)nullptr, B.nsolve, off, c, cstride, u);
  ktimer().end(s);
  RBWS_HIP(hipGetLastError());
}

Basis* rb_build(const Problem* P, const double* mu_train, int ntrain, int N, double snap_tol, int prec,
                int snap_maxit, int flags, hipStream_t s) {
  RBWS_REQUIRE(ntrain >= 1, RBWS_EINVAL, "empty training set");
  RBWS_REQUIRE(N >= 1 && N <= kMaxN, RBWS_EINVAL, "N must be in [1, 64]");
  RBWS_REQUIRE(N <= ntrain, RBWS_EINVAL, "N exceeds the training set");
  RBWS_REQUIRE(snap_tol > 0.0 && std::isfinite(snap_tol), RBWS_EINVAL, "snap_tol must be positive");
  RBWS_HIP(hipSetDevice(P->device));
  const int fe = (flags & RBWS_FLAG_FORCE_EXACT_DOTS) ? 1 : 0;
  const long long nd = P->ndof;
  const int Q = P->Q, dev = P->device;
  Basis* bs = new Basis();
  try {
    bs->prob = P;
    bs->Nmax = N;
    bs->Q = Q;
    bs->ndof = nd;
    bs->ntrain = ntrain;
    bs->AqN.assign((size_t)Q * N * N, 0.0);
    bs->fN.assign(N, 0.0);
    double* V = (double*)bs->V.get(sizeof(double) * N * nd, dev);
    DevBuf vbuf, wbuf, fbuf, scal, cbuf, redob;
    double* v = (double*)vbuf.get(sizeof(double) * nd, dev);
    double* W = (double*)wbuf.get(sizeof(double) * Q * nd, dev);
    double* f = (double*)fbuf.get(sizeof(double) * nd, dev);
    double* sc = (double*)scal.get(sizeof(double) * (kMaxN * kMaxQ + 8), dev);
    const long long rcap = std::max<long long>(kRedoCap, nd);
    Redo* redo = (Redo*)redob.get(sizeof(Redo) + sizeof(long long) * rcap, dev);
    const double h = 1.0 / (P->n + 1);
    fill64(f, nd, h * h, s);
    // residual decomposition: keep every W_(q,i) (at most 8 GB)
    const bool est = P->desc.f_kind == RBWS_F_ONE && (double)Q * N * nd * sizeof(double) <= 8e9;
    DevBuf wallb;
    double* Wall = est ? (double*)wallb.get(sizeof(double) * Q * N * nd, dev) : nullptr;
    const int QN = Q * N;
    if (est) {
      bs->G.assign((size_t)QN * QN, 0.0);
      bs->g.assign(QN, 0.0);
      pair_dots({f}, {f}, nd, sc, fe, dev, s);
      RBWS_HIP(hipMemcpyAsync(&bs->ff, sc, sizeof(double), hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
    }
    std::vector<const Problem*> probs{P};
    Batch snap, eq, tr;
    // A_q = A(theta = e_q): a batch of Q "solves" with unit theta vectors
    std::vector<double> eth((size_t)Q * Q, 0.0);
    for (int q = 0; q < Q; q++) eth[(size_t)q * Q + q] = 1.0;
    batch_setup(eq, probs, nullptr, Q, mu_train, P->p, s, eth.data());
    // training batch in chunks of at most `chunk` parameters
    const long long budget = 4LL << 30;  // bytes for the lifted training vectors
    int chunk = (int)std::max<long long>(1, std::min<long long>(ntrain, budget / (8 * nd)));
    const int stride = kMaxN;
    std::vector<double> delta(ntrain), hrow;
    int l = 0, nb = 0;
    for (;;) {
      // snapshot u(mu_l) by Alg. 1 from zero
      batch_setup(snap, probs, nullptr, 1, mu_train + (long long)l * P->p, P->p, s);
      double* x = (double*)snap.x.get(sizeof(double) * nd, dev);
      fill64(x, nd, 0.0, s);
      cg_fp64_run(snap, CgOpts{snap_tol, snap_maxit, prec, flags, 0}, s);
      RBWS_HIP(hipMemcpyAsync(v, x, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
      // two classical Gram-Schmidt passes
      for (int pass = 0; pass < 2 && nb > 0; pass++) {
        std::vector<const double*> xs, ys;
        for (int j = 0; j < nb; j++) {
          xs.push_back(V + (long long)j * nd);
          ys.push_back(v);
        }
        pair_dots(xs, ys, nd, sc, fe, dev, s);
        RBWS_HIP(hipMemsetAsync(redo, 0, sizeof(Redo), s));
        hipLaunchKernelGGL(k_gs_update, dim3(2048), dim3(256), 0, s, v, (const double*)V, (const double*)sc, nb,
                           nd, redo, fe, rcap);
        hipLaunchKernelGGL(k_gs_redo, dim3(1024), dim3(64), 0, s, v, (const double*)V, (const double*)sc, nb,
                           nd, (const Redo*)redo);
        RBWS_HIP(hipGetLastError());
      }
      pair_dots({v, x}, {v, x}, nd, sc + kMaxN * kMaxQ, fe, dev, s);
      double nn[2];
      RBWS_HIP(hipMemcpyAsync(nn, sc + kMaxN * kMaxQ, sizeof nn, hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
      const double nrm = std::sqrt(nn[0]), unrm = std::sqrt(nn[1]);
      if (!(nrm >= 1e-10 * unrm)) break;  // the snapshot adds nothing new
      RBWS_HIP(hipMemcpyAsync(sc + kMaxN * kMaxQ + 2, &nrm, sizeof(double), hipMemcpyHostToDevice, s));
      double* vn = V + (long long)nb * nd;
      hipLaunchKernelGGL(k_div, dim3(2048), dim3(256), 0, s, vn, (const double*)v,
                         (const double*)(sc + kMaxN * kMaxQ + 2), nd);
      bs->selected.push_back(l);
      // W_q = A_q v_n, then the new row/column of every A_q^N and f^N
      hipLaunchKernelGGL(k_copy_rep, dim3(2048), dim3(256), 0, s, W, (const double*)vn, nd, Q);
      {
        double* Wx = (double*)eq.x.get(sizeof(double) * Q * nd, dev);
        RBWS_HIP(hipMemcpyAsync(Wx, W, sizeof(double) * Q * nd, hipMemcpyDeviceToDevice, s));
        spmv_batch(eq, Wx, W, false, s);
      }
      std::vector<const double*> xs, ys;
      for (int q = 0; q < Q; q++)
        for (int i = 0; i <= nb; i++) {
          xs.push_back(V + (long long)i * nd);
          ys.push_back(W + (long long)q * nd);
        }
      xs.push_back(vn);
      ys.push_back(f);
      pair_dots(xs, ys, nd, sc, fe, dev, s);
      std::vector<double> hv(xs.size());
      RBWS_HIP(hipMemcpyAsync(hv.data(), sc, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < Q; q++)
        for (int i = 0; i <= nb; i++) {
          const double a = hv[(size_t)q * (nb + 1) + i];
          bs->AqN[((size_t)q * N + i) * N + nb] = a;
          bs->AqN[((size_t)q * N + nb) * N + i] = a;
        }
      bs->fN[nb] = hv.back();
      if (est) {  // new row and column of G and g: W_(q,nb) against every kept W and f
        for (int q = 0; q < Q; q++)
          RBWS_HIP(hipMemcpyAsync(Wall + ((long long)q * N + nb) * nd, W + (long long)q * nd,
                                  sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
        std::vector<const double*> ws, wt;
        for (int q = 0; q < Q; q++) {
          for (int q2 = 0; q2 < Q; q2++)
            for (int j = 0; j <= nb; j++) {
              ws.push_back(Wall + ((long long)q * N + nb) * nd);
              wt.push_back(Wall + ((long long)q2 * N + j) * nd);
            }
          ws.push_back(Wall + ((long long)q * N + nb) * nd);
          wt.push_back(f);
        }
        RBWS_SCRATCH(gdots);
        double* gdd = (double*)gdots.get(sizeof(double) * ws.size(), dev);
        pair_dots(ws, wt, nd, gdd, fe, dev, s);
        std::vector<double> gv(ws.size());
        RBWS_HIP(hipMemcpyAsync(gv.data(), gdd, sizeof(double) * gv.size(), hipMemcpyDeviceToHost, s));
        RBWS_HIP(hipStreamSynchronize(s));
        size_t o = 0;
        for (int q = 0; q < Q; q++) {
          const size_t r = (size_t)q * N + nb;
          for (int q2 = 0; q2 < Q; q2++)
            for (int j = 0; j <= nb; j++) {
              const size_t c2 = (size_t)q2 * N + j;
              bs->G[r * QN + c2] = gv[o];
              bs->G[c2 * QN + r] = gv[o];
              o++;
            }
          bs->g[r] = gv[o++];
        }
      }
      nb++;
      bs->N = nb;
      bs->upload(s);
      // indicator over the training set with nb basis vectors
      std::vector<const Basis*> bl{bs};
      for (int t0 = 0; t0 < ntrain; t0 += chunk) {
        const int cnt = std::min(chunk, ntrain - t0);
        batch_setup(tr, probs, nullptr, cnt, mu_train + (long long)t0 * P->p, P->p, s);
        double* cd = (double*)cbuf.get(sizeof(double) * stride * cnt, dev);
        RBWS_REQUIRE(rb_coeffs(tr, bl, cd, stride, fe, s) == 0, RBWS_ENUMERIC,
                     "reduced matrix not positive definite in the greedy");
        double* ux = (double*)tr.x.get(sizeof(double) * cnt * nd, dev);
        rb_lift_exact(tr, bl, cd, stride, ux, fe, s);
        resid_norms(tr, ux, delta.data() + t0, nullptr, nullptr, fe, s);
      }
      bs->hist.insert(bs->hist.end(), delta.begin(), delta.end());
      for (double dlt : delta) RBWS_REQUIRE(std::isfinite(dlt), RBWS_ENUMERIC, "non-finite indicator");
      if (nb == N) break;
      int best = 0;
      for (int t = 1; t < ntrain; t++)
        if (delta[t] > delta[best]) best = t;
      if (std::find(bs->selected.begin(), bs->selected.end(), best) != bs->selected.end()) break;
      l = best;
    }
    RBWS_REQUIRE(nb >= 1, RBWS_ENUMERIC, "the first snapshot is zero");
    const double* last = bs->hist.data() + (size_t)(nb - 1) * ntrain;
    bs->final_max = *std::max_element(last, last + ntrain);
    bs->est = est;
    bs->upload(s);
  } catch (...) {
    delete bs;
    throw;
  }
  return bs;
}

// ---------------------------------------------------------------------------
// residual of the reduced solution from the decomposition (one block per solve)
// ---------------------------------------------------------------------------
struct EstDev {
  const double* G;
  const double* g;
  double ff;
  int Q, ld, N, pad;
};

__global__ __launch_bounds__(256) void k_rb_est(const SolveDev* __restrict__ sd, const EstDev* __restrict__ ed,
                                                const double* __restrict__ theta, const double* __restrict__ c,
                                                int cstride, double* __restrict__ out) {
  __shared__ double y[kMaxQ * kMaxN];
  __shared__ double red[4][4];
  const int b = blockIdx.x;
  const EstDev E = ed[sd[b].prob];
  const int QN = E.Q * E.ld;
  for (int x = threadIdx.x; x < QN; x += blockDim.x) {
    const int q = x / E.ld, i = x - q * E.ld;
    y[x] = i < E.N ? theta[(long long)b * kMaxQ + q] * c[(long long)b * cstride + i] : 0.0;
  }
  __syncthreads();
  double quad = 0.0, mag = 0.0, lin = 0.0, maglin = 0.0;
  for (int r = threadIdx.x; r < QN; r += blockDim.x) {
    const double yr = y[r];
    if (yr == 0.0) continue;
    const double* Gr = E.G + (long long)r * QN;
    double acc = 0.0, am = 0.0;
    for (int k = 0; k < QN; k++) {
      const double gv = Gr[k];
      acc = __fma_rn(gv, y[k], acc);
      am = __fma_rn(fabs(gv), fabs(y[k]), am);
    }
    quad = __fma_rn(yr, acc, quad);
    mag = __fma_rn(fabs(yr), am, mag);
    lin = __fma_rn(yr, E.g[r], lin);
    maglin = __fma_rn(fabs(yr), fabs(E.g[r]), maglin);
  }
  for (int m = 32; m >= 1; m >>= 1) {
    quad += __shfl_xor(quad, m, 64);
    mag += __shfl_xor(mag, m, 64);
    lin += __shfl_xor(lin, m, 64);
    maglin += __shfl_xor(maglin, m, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = quad;
    red[w][1] = mag;
    red[w][2] = lin;
    red[w][3] = maglin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < (int)(blockDim.x >> 6); v++)
      for (int e = 0; e < 4; e++) t[e] += red[v][e];
    out[2 * b] = (E.ff - 2.0 * t[2]) + t[0];
    out[2 * b + 1] = (E.ff + 2.0 * t[3]) + t[1];
  }
}

int rb_resid_estimate(Batch& B, const std::vector<const Basis*>& bases, const double* c, int cstride, double* rel,
                      hipStream_t s) {
  const int ns = B.nsolve;
  if (ns == 0) return 0;
  std::vector<EstDev> eh(B.nprob);
  for (int q = 0; q < B.nprob; q++) {
    const Basis* bs = bases[q];
    RBWS_REQUIRE(bs != nullptr && bs->est, RBWS_ESTATE, "the basis has no residual decomposition");
    RBWS_REQUIRE(bs->Q <= kMaxQ && bs->Nmax <= kMaxN, RBWS_EINVAL, "basis too large for the estimator");
    eh[q] = EstDev{(const double*)bs->G_d.ptr, (const double*)bs->g_d.ptr, bs->ff, bs->Q, bs->Nmax, bs->N, 0};
  }
  RBWS_SCRATCH(edb);
  RBWS_SCRATCH(outb);
  EstDev* ed = (EstDev*)edb.get(sizeof(EstDev) * eh.size(), B.device);
  double* o = (double*)outb.get(sizeof(double) * 2 * ns, B.device);
  RBWS_HIP(hipMemcpyAsync(ed, eh.data(), sizeof(EstDev) * eh.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_rb_est, dim3(ns), dim3(256), 0, s, (const SolveDev*)B.sd.ptr, (const EstDev*)ed,
                     (const double*)B.theta.ptr, c, cstride, o);
  RBWS_HIP(hipGetLastError());
  std::vector<double> h(2 * (size_t)ns);
  RBWS_HIP(hipMemcpyAsync(h.data(), o, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  int bad = 0;
  for (int b = 0; b < ns; b++) {
    const double rr = h[2 * b], mag = h[2 * b + 1], ff = eh[B.sd_h[b].prob].ff;
    if (std::isfinite(rr) && !(rr >= 1e-8 * mag)) bad++;
    rel[b] = std::isfinite(rr) ? std::sqrt(std::max(rr, 0.0) / ff) : std::nan("");
  }
  return bad;
}

// ---------------------------------------------------------------------------
// save / load: a small binary file (little-endian host layout)
// ---------------------------------------------------------------------------
struct BasisHeader {
  char magic[8];
  int n, kind, nblocks, f_kind;
  int Nmax, N, Q, ntrain;
  long long ndof;
  double final_max;
  int blocks[6 * 32];
};

void basis_save(const Basis* b, const char* path) {
  RBWS_REQUIRE(b->kind == 0, RBWS_EINVAL, "saving an L1ROC basis is not supported");
  RBWS_REQUIRE(b && path, RBWS_EINVAL, "NULL argument");
  BasisHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "RBWSBAS1", 8);
  const Problem* P = b->prob;
  h.n = P->n;
  h.kind = P->desc.kind;
  h.nblocks = P->desc.nblocks;
  h.f_kind = P->desc.f_kind;
  h.Nmax = b->Nmax;
  h.N = b->N;
  h.Q = b->Q;
  h.ntrain = b->ntrain;
  h.ndof = b->ndof;
  h.final_max = b->final_max;
  for (size_t i = 0; i < P->blocks.size() && i < 6 * 32; i++) h.blocks[i] = P->blocks[i];
  std::vector<double> V((size_t)b->N * b->ndof);
  RBWS_HIP(hipSetDevice(P->device));
  RBWS_HIP(hipMemcpy(V.data(), b->V.ptr, sizeof(double) * V.size(), hipMemcpyDeviceToHost));
  FILE* fp = std::fopen(path, "wb");
  RBWS_REQUIRE(fp != nullptr, RBWS_EINVAL, std::string("cannot open ") + path);
  bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
  ok = ok && std::fwrite(b->AqN.data(), sizeof(double), b->AqN.size(), fp) == b->AqN.size();
  ok = ok && std::fwrite(b->fN.data(), sizeof(double), b->fN.size(), fp) == b->fN.size();
  ok = ok && std::fwrite(b->selected.data(), sizeof(int), b->selected.size(), fp) == b->selected.size();
  ok = ok && std::fwrite(b->hist.data(), sizeof(double), b->hist.size(), fp) == b->hist.size();
  ok = ok && std::fwrite(V.data(), sizeof(double), V.size(), fp) == V.size();
  ok = (std::fclose(fp) == 0) && ok;
  RBWS_REQUIRE(ok, RBWS_EINVAL, std::string("write failed: ") + path);
}

Basis* basis_load(const Problem* P, const char* path, hipStream_t s) {
  RBWS_REQUIRE(P && path, RBWS_EINVAL, "NULL argument");
  FILE* fp = std::fopen(path, "rb");
  RBWS_REQUIRE(fp != nullptr, RBWS_EINVAL, std::string("cannot open ") + path);
  BasisHeader h;
  Basis* b = nullptr;
  try {
    RBWS_REQUIRE(std::fread(&h, sizeof h, 1, fp) == 1 && std::memcmp(h.magic, "RBWSBAS1", 8) == 0,
                 RBWS_EINVAL, "not a basis file");
    RBWS_REQUIRE(h.n == P->n && h.kind == P->desc.kind && h.nblocks == P->desc.nblocks &&
                     h.f_kind == P->desc.f_kind && h.Q == P->Q && h.ndof == P->ndof,
                 RBWS_EINVAL, "basis file belongs to another problem");
    for (size_t i = 0; i < P->blocks.size(); i++)
      RBWS_REQUIRE(h.blocks[i] == P->blocks[i], RBWS_EINVAL, "basis file belongs to another problem");
    RBWS_REQUIRE(h.N >= 1 && h.N <= h.Nmax && h.Nmax <= kMaxN && h.ntrain >= 1, RBWS_EINVAL, "corrupt basis file");
    b = new Basis();
    b->prob = P;
    b->Nmax = h.Nmax;
    b->N = h.N;
    b->Q = h.Q;
    b->ndof = h.ndof;
    b->ntrain = h.ntrain;
    b->final_max = h.final_max;
    b->AqN.resize((size_t)h.Q * h.Nmax * h.Nmax);
    b->fN.resize(h.Nmax);
    b->selected.resize(h.N);
    b->hist.resize((size_t)h.N * h.ntrain);
    std::vector<double> V((size_t)h.N * h.ndof);
    bool ok = std::fread(b->AqN.data(), sizeof(double), b->AqN.size(), fp) == b->AqN.size();
    ok = ok && std::fread(b->fN.data(), sizeof(double), b->fN.size(), fp) == b->fN.size();
    ok = ok && std::fread(b->selected.data(), sizeof(int), b->selected.size(), fp) == b->selected.size();
    ok = ok && std::fread(b->hist.data(), sizeof(double), b->hist.size(), fp) == b->hist.size();
    ok = ok && std::fread(V.data(), sizeof(double), V.size(), fp) == V.size();
    RBWS_REQUIRE(ok, RBWS_EINVAL, "truncated basis file");
    RBWS_HIP(hipSetDevice(P->device));
    double* d = (double*)b->V.get(sizeof(double) * h.Nmax * h.ndof, P->device);
    RBWS_HIP(hipMemcpy(d, V.data(), sizeof(double) * V.size(), hipMemcpyHostToDevice));
    b->upload(s);
  } catch (...) {
    std::fclose(fp);
    delete b;
    throw;
  }
  std::fclose(fp);
  return b;
}

// ---------------------------------------------------------------------------
// L1-based reduced over-collocation, L1ROC (Sec. 3.1, Alg. 4)
// ---------------------------------------------------------------------------
// The basis vectors are DEIM-normalised (w_j(x_j) = 1 and w_j(x_i) = 0 for
// i < j at the snapshot points).  Online, c minimises ||P (f - A(mu) W c)||_2
// over the collocation points by Householder QR, one wave per parameter:
// every inner product is correctly rounded and every update is a separately
// rounded product and difference, so the result is that of the sequential
// definition, bit for bit.  The greedy's indicator is ||T c||_1 (W = U T).

constexpr int kL1MaxM = 2 * kL1MaxN - 1;  // the first step adds one point, every later step at most two

struct L1Dev {           // per solve
  const double* W;       // nb x ndof
  const long long* pts;  // npts collocation points
  const double* T;       // ld x ld, or null
  int nb, npts, ld, pad;
};

struct L1Shared {
  double A[kL1MaxM * kL1MaxN];
  double b[kL1MaxM];
  double c[kL1MaxN];
  XAcc xa;
  uint32_t dig[XA_WORDS];
  double val;
  int ok;
};

// (A(mu) x) at one unknown: coefficients from the solve's class table, the
// operations and order of the sweeps (d x, then fma over x-, x+, y-, y+, z-, z+)
__device__ double point_apply(const GridDev& g, const double* kt, const double* x, long long pt) {
  const int n = g.n;
  const long long n2 = (long long)n * n;
  const int i = (int)(pt % n) + 1, j = (int)((pt / n) % n) + 1, k = (int)(pt / n2) + 1;
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  const int oY = g.ndir == 3 ? g.nclass : 0, oZ = g.ndir == 3 ? 2 * g.nclass : 0;
  const int cxn = g.code[0][0][i - 1], cxm = g.code[0][1][i - 1], cxp = g.code[0][1][i];
  const int cyn = g.code[1][0][j - 1], cym = g.code[1][1][j - 1], cyp = g.code[1][1][j];
  const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
  const double c0 = kt[(cxm * N1 + cyn) * N2 + czn], c1 = kt[(cxp * N1 + cyn) * N2 + czn];
  const double c2 = kt[oY + (cxn * N1 + cym) * N2 + czn], c3 = kt[oY + (cxn * N1 + cyp) * N2 + czn];
  const double c4 = kt[oZ + (cxn * N1 + cyn) * N2 + czm], c5 = kt[oZ + (cxn * N1 + cyn) * N2 + czp];
  const double d = ((((c0 + c1) + c2) + c3) + c4) + c5;
  double acc = d * x[pt];
  if (i > 1) acc = __fma_rn(-c0, x[pt - 1], acc);
  if (i < n) acc = __fma_rn(-c1, x[pt + 1], acc);
  if (j > 1) acc = __fma_rn(-c2, x[pt - n], acc);
  if (j < n) acc = __fma_rn(-c3, x[pt + n], acc);
  if (k > 1) acc = __fma_rn(-c4, x[pt - n2], acc);
  if (k < n) acc = __fma_rn(-c5, x[pt + n2], acc);
  return acc;
}

// Collocation least squares of one solve per 64-thread block, right-hand side
// f_h(mu) at the collocation points (the M point evaluations that replace the
// projection V^T f(mu) for a parameter-dependent source); optionally the L1
// indicator sum_i |sum_{j>=i} T_ij c_j|.
__global__ __launch_bounds__(64) void k_l1_lsq(const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                               const double* __restrict__ kap, const L1Dev* __restrict__ l1,
                                               double* __restrict__ cout, int cstride, double* __restrict__ delta,
                                               int* bad, int force_exact) {
  __shared__ L1Shared sh;
  const int b = blockIdx.x, lane = threadIdx.x;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const L1Dev L = l1[b];
  const int nb = L.nb, M = L.npts;
  const long long nd = P.g.ndof;
  const double* kt = kap + S.kap_off;
  for (int e = lane; e < M * nb; e += 64) {
    const int i = e / nb, j = e - i * nb;
    sh.A[i * kL1MaxN + j] = point_apply(P.g, kt, L.W + (long long)j * nd, L.pts[i]);
  }
  for (int i = lane; i < M; i += 64) {
    const long long pt = L.pts[i];
    const int n = P.g.n;
    sh.b[i] = fval(P, S, (int)(pt % n) + 1, (int)((pt / n) % n) + 1, (int)(pt / ((long long)n * n)) + 1);
  }
  __syncthreads();
  int fail = 0;
  for (int k = 0; k < nb; k++) {
    CrAcc a = cr_zero();
    for (int i = k + lane; i < M; i += 64) cr_add_prod(a, sh.A[i * kL1MaxN + k], sh.A[i * kL1MaxN + k]);
    const double n2v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      for (int i = k + lane; i < M; i += 64) xa_add_prod(x, sh.A[i * kL1MaxN + k], sh.A[i * kL1MaxN + k]);
    });
    const double nrm = sqrt(n2v);
    if (!(nrm > 0.0)) {
      fail = 1;
      break;
    }
    const double akk = sh.A[k * kL1MaxN + k];
    const double alpha = akk > 0.0 ? -nrm : nrm;
    const double vk = akk - alpha;
    const double vtv = 2.0 * nrm * (nrm + fabs(akk));
    for (int j = k + 1; j <= nb; j++) {  // j == nb: the right-hand side
      auto at = [&](int i) -> double& { return j < nb ? sh.A[i * kL1MaxN + j] : sh.b[i]; };
      CrAcc d = cr_zero();
      if (lane == 0) cr_add_prod(d, vk, at(k));
      for (int i = k + 1 + lane; i < M; i += 64) cr_add_prod(d, sh.A[i * kL1MaxN + k], at(i));
      const double dv = wave_sum(sh, d, force_exact, [&](XAcc* x) {
        if (lane == 0) xa_add_prod(x, vk, at(k));
        for (int i = k + 1 + lane; i < M; i += 64) xa_add_prod(x, sh.A[i * kL1MaxN + k], at(i));
      });
      const double t = 2.0 * dv / vtv;
      if (lane == 0) at(k) = at(k) - t * vk;
      for (int i = k + 1 + lane; i < M; i += 64) at(i) = at(i) - t * sh.A[i * kL1MaxN + k];
      __syncthreads();
    }
    if (lane == 0) sh.A[k * kL1MaxN + k] = alpha;
    __syncthreads();
  }
  if (fail) {
    if (lane == 0) {
      atomicAdd(bad, 1);
      if (delta) delta[b] = __builtin_nan("");
    }
    for (int j = lane; j < cstride; j += 64) cout[(long long)b * cstride + j] = __builtin_nan("");
    return;
  }
  for (int k = nb - 1; k >= 0; k--) {  // R c = Q^T b
    CrAcc a = cr_zero();
    if (lane == 0) cr_add(a, sh.b[k]);
    for (int j = k + 1 + lane; j < nb; j += 64) cr_add_prod(a, -sh.A[k * kL1MaxN + j], sh.c[j]);
    const double v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane == 0) xa_add(x, sh.b[k]);
      for (int j = k + 1 + lane; j < nb; j += 64) xa_add_prod(x, -sh.A[k * kL1MaxN + j], sh.c[j]);
    });
    if (lane == 0) sh.c[k] = v / sh.A[k * kL1MaxN + k];
    __syncthreads();
  }
  for (int j = lane; j < cstride; j += 64) cout[(long long)b * cstride + j] = j < nb ? sh.c[j] : 0.0;
  if (delta && L.T) {
    double cu = 0.0;  // lane i: |(T c)_i|
    for (int i = 0; i < nb; i++) {
      CrAcc a = cr_zero();
      if (lane >= i && lane < nb) cr_add_prod(a, L.T[(long long)i * L.ld + lane], sh.c[lane]);
      const double v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
        if (lane >= i && lane < nb) xa_add_prod(x, L.T[(long long)i * L.ld + lane], sh.c[lane]);
      });
      if (lane == i) cu = fabs(v);
    }
    CrAcc a = cr_zero();
    if (lane < nb) cr_add(a, cu);
    const double sum = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane < nb) xa_add(x, cu);
    });
    if (lane == 0) delta[b] = sum;
  }
}

struct WaveShared {
  XAcc xa;
  uint32_t dig[XA_WORDS];
  double val;
  int ok;
  double c[kL1MaxN + 1];
};

// DEIM interpolation coefficients of x against the nb vectors B at their
// points: sum_{j<=i} B_j(x_i) c_j = x(x_i) with B_i(x_i) = 1 (forward
// substitution, each entry correctly rounded); one 64-thread block
__global__ __launch_bounds__(64) void k_deim_coef(const double* __restrict__ B, long long nd,
                                                  const long long* __restrict__ pts, int nb,
                                                  const double* __restrict__ x, double* __restrict__ c,
                                                  int force_exact) {
  __shared__ WaveShared sh;
  const int lane = threadIdx.x;
  for (int i = 0; i < nb; i++) {
    const long long pi = pts[i];
    CrAcc a = cr_zero();
    if (lane == 0) cr_add(a, x[pi]);
    for (int j = lane; j < i; j += 64) cr_add_prod(a, -B[(long long)j * nd + pi], sh.c[j]);
    const double v = wave_sum(sh, a, force_exact, [&](XAcc* xa) {
      if (lane == 0) xa_add(xa, x[pi]);
      for (int j = lane; j < i; j += 64) xa_add_prod(xa, -B[(long long)j * nd + pi], sh.c[j]);
    });
    if (lane == 0) sh.c[i] = v;
    __syncthreads();
  }
  for (int j = lane; j < nb; j += 64) c[j] = sh.c[j];
}

// T[i][nb] = (-sum_{j=i}^{nb-1} c_j T[i][j]) / s for i < nb, T[nb][nb] = 1 / s
__global__ __launch_bounds__(64) void k_l1_tcol(double* __restrict__ T, int ld, const double* __restrict__ c,
                                                int nb, const double* __restrict__ sp, int force_exact) {
  __shared__ WaveShared sh;
  const int lane = threadIdx.x;
  const double s = *sp;
  for (int i = 0; i < nb; i++) {
    CrAcc a = cr_zero();
    if (lane >= i && lane < nb) cr_add_prod(a, -c[lane], T[(long long)i * ld + lane]);
    const double v = wave_sum(sh, a, force_exact, [&](XAcc* x) {
      if (lane >= i && lane < nb) xa_add_prod(x, -c[lane], T[(long long)i * ld + lane]);
    });
    if (lane == 0) T[(long long)i * ld + nb] = v / s;
    __syncthreads();
  }
  if (lane == 0) T[(long long)nb * ld + nb] = 1.0 / s;
}

__global__ void k_zero_at(double* __restrict__ r, const long long* __restrict__ pts, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) r[pts[i]] = 0.0;
}

// largest |r_k|, lowest index on ties: per-block candidates, then one block
struct ValIdx {
  double v;
  long long i;
};
__device__ __forceinline__ ValIdx vi_better(ValIdx a, ValIdx b) {
  return (b.v > a.v || (b.v == a.v && b.i >= 0 && (a.i < 0 || b.i < a.i))) ? b : a;
}
__device__ ValIdx vi_block(ValIdx m) {
  __shared__ ValIdx w[4];
  for (int o = 32; o >= 1; o >>= 1) {
    ValIdx t{__shfl_xor(m.v, o, 64), __shfl_xor(m.i, o, 64)};
    m = vi_better(m, t);
  }
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
  __syncthreads();
  m = w[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); k++) m = vi_better(m, w[k]);
  __syncthreads();
  return m;
}
__global__ __launch_bounds__(256) void k_absmax_part(const double* __restrict__ r, long long nd,
                                                     ValIdx* __restrict__ part) {
  ValIdx m{0.0, -1};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nd; k += (long long)gridDim.x * blockDim.x) {
    const double a = fabs(r[k]);
    if (a > m.v) m = ValIdx{a, k};  // ascending k per thread: the first maximiser
  }
  m = vi_block(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}
// part[0] <- the overall winner, with the signed value r[i] in out[0] and 1 / r[i] unused
__global__ __launch_bounds__(256) void k_absmax_final(ValIdx* __restrict__ part, int nparts,
                                                      const double* __restrict__ r, double* __restrict__ sval) {
  ValIdx m{0.0, -1};
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) m = vi_better(m, part[k]);
  m = vi_block(m);
  if (threadIdx.x == 0) {
    part[0] = m;
    *sval = m.i >= 0 ? r[m.i] : 0.0;
  }
}

__global__ void k_neg(double* __restrict__ out, const double* __restrict__ in, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = -in[i];
}
// r = f_h(mu) - A u of the batch's first solve
__global__ void k_rhs_minus(double* __restrict__ r, const double* __restrict__ au, const ProbDev* __restrict__ pd,
                            const SolveDev* __restrict__ sd, long long nd) {
  const SolveDev S = sd[0];
  const ProbDev& P = pd[S.prob];
  const int n = P.g.n;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nd; c += (long long)gridDim.x * blockDim.x)
    r[c] = fval(P, S, (int)(c % n) + 1, (int)((c / n) % n) + 1, (int)(c / ((long long)n * n)) + 1) - au[c];
}

static int l1roc_coeffs(Batch& B, const std::vector<const Basis*>& bases, double* c, int cstride,
                        double* delta, int force_exact, hipStream_t s) {
  const int ns = B.nsolve;
  std::vector<L1Dev> h(ns);
  for (int b = 0; b < ns; b++) {
    const Basis* bs = bases[B.sd_h[b].prob];
    RBWS_REQUIRE(bs != nullptr && bs->kind == 1, RBWS_ESTATE, "an L1ROC basis is required");
    RBWS_REQUIRE(bs->prob == B.probs[B.sd_h[b].prob], RBWS_EINVAL, "basis belongs to another problem");
    RBWS_REQUIRE(bs->N <= cstride, RBWS_EINVAL, "coefficient stride too small");
    RBWS_REQUIRE(bs->N <= kL1MaxN && (int)bs->pts.size() <= kL1MaxM && (int)bs->pts.size() >= bs->N,
                 RBWS_EINVAL, "L1ROC basis outside the kernel's limits");
    h[b] = L1Dev{(const double*)bs->V.ptr, (const long long*)bs->pts_d.ptr, (const double*)bs->T_d.ptr, bs->N,
                 (int)bs->pts.size(), bs->Nmax, 0};
  }
  RBWS_SCRATCH(l1d);
  RBWS_SCRATCH(badb);
  L1Dev* d = (L1Dev*)l1d.get(sizeof(L1Dev) * ns, B.device);
  int* bad = (int*)badb.get(sizeof(int), B.device);
  RBWS_HIP(hipMemcpyAsync(d, h.data(), sizeof(L1Dev) * ns, hipMemcpyHostToDevice, s));
  RBWS_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  ktimer().begin(s, KK_COEF);
  hipLaunchKernelGGL(k_l1_lsq, dim3(ns), dim3(64), 0, s, (const SolveDev*)B.sd.ptr, (const ProbDev*)B.pd.ptr,
                     (const double*)B.kap64.ptr, (const L1Dev*)d, c, cstride, delta, bad, force_exact);
  ktimer().end(s);
  RBWS_HIP(hipGetLastError());
  int hb = 0;
  RBWS_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  return hb;
}

// one DEIM step of x against the nb vectors in Bv (points pt_d / pt): the
// new normalised vector goes to out; returns the new point or -1
static long long deim_gpu(const double* Bv, int nb, const long long* pt_d, long long nd, const double* x,
                          double* out, double* coef, double* sval, double* sc_host, Redo* redo, long long rcap,
                          ValIdx* part, int nparts, int fe, hipStream_t s) {
  hipLaunchKernelGGL(k_deim_coef, dim3(1), dim3(64), 0, s, Bv, nd, pt_d, nb, x, coef, fe);
  RBWS_HIP(hipMemcpyAsync(out, x, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
  if (nb > 0) {
    RBWS_HIP(hipMemsetAsync(redo, 0, sizeof(Redo), s));
    hipLaunchKernelGGL(k_gs_update, dim3(2048), dim3(256), 0, s, out, Bv, (const double*)coef, nb, nd, redo, fe, rcap);
    hipLaunchKernelGGL(k_gs_redo, dim3(1024), dim3(64), 0, s, out, Bv, (const double*)coef, nb, nd,
                       (const Redo*)redo);
    hipLaunchKernelGGL(k_zero_at, dim3(1), dim3(64), 0, s, out, pt_d, nb);
  }
  hipLaunchKernelGGL(k_absmax_part, dim3(nparts), dim3(256), 0, s, (const double*)out, nd, part);
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, s, part, nparts, (const double*)out, sval);
  RBWS_HIP(hipGetLastError());
  ValIdx w;
  RBWS_HIP(hipMemcpyAsync(&w, part, sizeof(ValIdx), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipMemcpyAsync(sc_host, sval, sizeof(double), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  if (w.i < 0) return -1;
  hipLaunchKernelGGL(k_div, dim3(2048), dim3(256), 0, s, out, (const double*)out, (const double*)sval, nd);
  RBWS_HIP(hipGetLastError());
  return w.i;
}

Basis* rb_build_l1roc(const Problem* P, const double* mu_train, int ntrain, int N, double snap_tol, int prec,
                      int snap_maxit, int flags, hipStream_t s) {
  RBWS_REQUIRE(ntrain >= 1, RBWS_EINVAL, "empty training set");
  RBWS_REQUIRE(N >= 1 && N <= kL1MaxN, RBWS_EINVAL, "N must be in [1, 60] for L1ROC");
  RBWS_REQUIRE(N <= ntrain, RBWS_EINVAL, "N exceeds the training set");
  RBWS_REQUIRE(snap_tol > 0.0 && std::isfinite(snap_tol), RBWS_EINVAL, "snap_tol must be positive");
  RBWS_HIP(hipSetDevice(P->device));
  const int fe = (flags & RBWS_FLAG_FORCE_EXACT_DOTS) ? 1 : 0;
  const long long nd = P->ndof;
  const int dev = P->device;
  Basis* bs = new Basis();
  try {
    bs->prob = P;
    bs->kind = 1;
    bs->Nmax = N;
    bs->Q = P->Q;
    bs->ndof = nd;
    bs->ntrain = ntrain;
    bs->T.assign((size_t)N * N, 0.0);
    double* W = (double*)bs->V.get(sizeof(double) * N * nd, dev);
    DevBuf rbuf, ubuf, resb, aub, cbuf, scal, redob, partb, xrb, tdb, dlb;
    double* R = (double*)rbuf.get(sizeof(double) * N * nd, dev);
    double* r = (double*)resb.get(sizeof(double) * nd, dev);
    double* au = (double*)aub.get(sizeof(double) * nd, dev);
    double* sc = (double*)scal.get(sizeof(double) * (4 * kL1MaxN + 8), dev);
    double* coef = sc;                  // DEIM coefficients
    double* cl = sc + kL1MaxN;          // collocation coefficients at the chosen parameter
    double* ncl = sc + 2 * kL1MaxN;     // their negation (lift through the Gram-Schmidt update)
    double* sval = sc + 3 * kL1MaxN;    // DEIM scale
    const long long rcap = std::max<long long>(kRedoCap, nd);
    Redo* redo = (Redo*)redob.get(sizeof(Redo) + sizeof(long long) * rcap, dev);
    const int nparts = 1024;
    ValIdx* part = (ValIdx*)partb.get(sizeof(ValIdx) * nparts, dev);
    long long* xs_d = (long long*)ubuf.get(sizeof(long long) * kL1MaxN, dev);
    long long* xr_d = (long long*)xrb.get(sizeof(long long) * kL1MaxN, dev);
    double* T_d = (double*)tdb.get(sizeof(double) * N * N, dev);
    RBWS_HIP(hipMemsetAsync(T_d, 0, sizeof(double) * N * N, s));
    double* delta_d = (double*)dlb.get(sizeof(double) * ntrain, dev);
    std::vector<const Problem*> probs{P};
    Batch snap, one, tr;
    batch_setup(tr, probs, nullptr, ntrain, mu_train, P->p, s);
    std::vector<double> delta(ntrain);
    auto snapshot = [&](int l) -> double* {
      batch_setup(snap, probs, nullptr, 1, mu_train + (long long)l * P->p, P->p, s);
      double* x = (double*)snap.x.get(sizeof(double) * nd, dev);
      fill64(x, nd, 0.0, s);
      cg_fp64_run(snap, CgOpts{snap_tol, snap_maxit, prec, flags, 0}, s);
      return x;
    };
    auto sync_points = [&]() {
      std::vector<long long> all(bs->xs);
      all.insert(all.end(), bs->xr.begin(), bs->xr.end());
      std::sort(all.begin(), all.end());
      all.erase(std::unique(all.begin(), all.end()), all.end());
      bs->pts = all;
      RBWS_HIP(hipMemcpyAsync(xs_d, bs->xs.data(), sizeof(long long) * bs->xs.size(), hipMemcpyHostToDevice, s));
      if (!bs->xr.empty())
        RBWS_HIP(hipMemcpyAsync(xr_d, bs->xr.data(), sizeof(long long) * bs->xr.size(), hipMemcpyHostToDevice, s));
      RBWS_HIP(hipMemcpyAsync(T_d, bs->T.data(), sizeof(double) * N * N, hipMemcpyHostToDevice, s));
      bs->upload(s);
    };
    std::vector<const Basis*> bl{bs};
    double shost = 0.0;
    // first snapshot
    {
      const double* x = snapshot(0);
      const long long pt = deim_gpu(W, 0, xs_d, nd, x, W, coef, sval, &shost, redo, rcap, part, nparts, fe, s);
      RBWS_REQUIRE(pt >= 0, RBWS_ENUMERIC, "the first snapshot is zero");
      bs->T[0] = 1.0 / shost;
      bs->xs.push_back(pt);
      bs->selected.push_back(0);
      bs->N = 1;
      sync_points();
    }
    for (;;) {
      const int nb = bs->N;
      RBWS_REQUIRE(l1roc_coeffs(tr, bl, (double*)cbuf.get(sizeof(double) * kL1MaxN * ntrain, dev), kL1MaxN,
                                delta_d, fe, s) == 0,
                   RBWS_ENUMERIC, "collocation least squares broke down in the greedy");
      RBWS_HIP(hipMemcpyAsync(delta.data(), delta_d, sizeof(double) * ntrain, hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
      bs->hist.insert(bs->hist.end(), delta.begin(), delta.end());
      if (nb == N) break;
      int best = 0;
      for (int t = 1; t < ntrain; t++)
        if (delta[t] > delta[best]) best = t;
      if (std::find(bs->selected.begin(), bs->selected.end(), best) != bs->selected.end()) break;
      const double* mul = mu_train + (long long)best * P->p;
      // residual of the current approximation at the chosen parameter
      batch_setup(one, probs, nullptr, 1, mul, P->p, s);
      RBWS_REQUIRE(l1roc_coeffs(one, bl, cl, kL1MaxN, nullptr, fe, s) == 0, RBWS_ENUMERIC,
                   "collocation least squares broke down in the greedy");
      hipLaunchKernelGGL(k_neg, dim3(1), dim3(64), 0, s, ncl, (const double*)cl, nb);
      RBWS_HIP(hipMemsetAsync(au, 0, sizeof(double) * nd, s));  // u = 0 - sum (-c_j) w_j
      RBWS_HIP(hipMemsetAsync(redo, 0, sizeof(Redo), s));
      hipLaunchKernelGGL(k_gs_update, dim3(2048), dim3(256), 0, s, au, (const double*)W, (const double*)ncl, nb,
                         nd, redo, fe, rcap);
      hipLaunchKernelGGL(k_gs_redo, dim3(1024), dim3(64), 0, s, au, (const double*)W, (const double*)ncl, nb, nd,
                         (const Redo*)redo);
      double* ux = (double*)one.x.get(sizeof(double) * nd, dev);
      RBWS_HIP(hipMemcpyAsync(ux, au, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
      spmv_batch(one, ux, au, false, s);
      hipLaunchKernelGGL(k_rhs_minus, dim3(2048), dim3(256), 0, s, r, (const double*)au, (const ProbDev*)one.pd.ptr,
                         (const SolveDev*)one.sd.ptr, nd);
      RBWS_HIP(hipGetLastError());
      // the snapshot's DEIM step
      const double* x = snapshot(best);
      const long long pt = deim_gpu(W, nb, xs_d, nd, x, W + (long long)nb * nd, coef, sval, &shost, redo, rcap, part,
                                    nparts, fe, s);
      if (pt < 0) break;
      hipLaunchKernelGGL(k_l1_tcol, dim3(1), dim3(64), 0, s, T_d, N, (const double*)coef, nb,
                         (const double*)sval, fe);
      RBWS_HIP(hipGetLastError());
      RBWS_HIP(hipMemcpyAsync(bs->T.data(), T_d, sizeof(double) * N * N, hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
      bs->xs.push_back(pt);
      // the residual's DEIM step adds a second point
      const int nr = (int)bs->xr.size();
      const long long ptr = deim_gpu(R, nr, xr_d, nd, r, R + (long long)nr * nd, coef, sval, &shost, redo, rcap, part,
                                     nparts, fe, s);
      if (ptr >= 0) bs->xr.push_back(ptr);
      bs->selected.push_back(best);
      bs->N = nb + 1;
      sync_points();
    }
    const double* last = bs->hist.data() + (size_t)(bs->N - 1) * ntrain;
    bs->final_max = *std::max_element(last, last + ntrain);
    bs->upload(s);
  } catch (...) {
    delete bs;
    throw;
  }
  return bs;
}

}  // namespace rbws
