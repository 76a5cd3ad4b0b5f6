// ir.hip -- FP32-inner / FP64-outer iterative refinement on gfx950.
//
// Not part of the paper's method (which states no precision); an addition that
// keeps the final accuracy of the FP64 system while the Krylov iterations move
// half the bytes.  Per solve:
//   outer pass (FP64): u <- u + 2^e d (the previous inner correction),
//                      r = f - A u, test ||r|| <= tol ||f||,
//                      b = fl32(r * 2^-e') with 2^e' a running estimate of ||r||
//   inner solve (FP32): PCG (Alg. 1 with P = I or Jacobi) on A32 d = b from
//                      d = 0, face coefficients rounded once to FP32, inner
//                      products accumulated in FP64, until ||r_in|| <= eta ||b||
//                      or inner_max iterations.
// CG is invariant under scaling the right-hand side by a power of two, so the
// choice of e' only keeps FP32 values away from overflow and underflow.  The
// outer pass reads u and d at the neighbours of each point to form the updated
// u there, so it writes the new u into the other of two buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "fast.hpp"

namespace rbws {

struct IrPart {
  CrAcc rr, ff;
  double g[3];
  double pad;
};

// Outer pass (FP64) of every solve whose mode is RESID: u_new = u + upd d,
// r = f - A64 u_new, b = fl32(r * scale) into r32, and the norms.
__global__ __launch_bounds__(256) void k_ir_outer(const int2* __restrict__ items, int per, int nitems,
                                                  const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                  const IrState* __restrict__ st, const double* __restrict__ kap64,
                                                  const float* __restrict__ kap32, double* __restrict__ u0,
                                                  double* __restrict__ u1, const float* __restrict__ d,
                                                  float* __restrict__ r, IrPart* __restrict__ part, int ktab) {
  extern __shared__ double lds[];
  __shared__ double redd[4][3];
  __shared__ CrAcc redc[4];
  const int item = item_of(blockIdx.x, per);
  if (item >= nitems) return;
  const int2 it = items[item];
  const int b = it.x;
  if (st[b].mode != MODE_RESID) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const GridDev& g = P.g;
  const int ntab = g.ndir * g.nclass;
  double* k64 = lds;
  float* k32 = reinterpret_cast<float*>(lds + ktab);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) {
    k32[e] = kap32[S.kap_off + e];
    k64[e] = kap64[S.kap_off + e];
  }
  __syncthreads();
  QuadGeo G;
  quad_geo(G, P, it.y);
  const int n = g.n;
  const long long n2 = (long long)n * n;
  const IrState& s = st[b];
  const int prec = s.prec, first = s.first;
  const double upd = s.upd, scale = s.scale;
  double g0 = 0.0, g1 = 0.0;
  CrAcc arr = cr_zero(), aff = cr_zero();
  const float* D = d + S.off;
  float* R = r + S.off;
  const double* Us = (s.cur ? u1 : u0) + S.off;
  double* Ud = (s.cur ? u0 : u1) + S.off;
  auto un = [&](long long e) { return upd != 0.0 ? __fma_rn(upd, (double)D[e], Us[e]) : Us[e]; };
  for (int k = G.kb; k <= G.ke; k++) {
    const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (e >= G.nv) continue;
      const int i = G.i + e, j = G.j;
      const long long c = vidx(n, i, j, k);
      double kd[6];
      float kk[6];
      quad_kappa<double>(G, k64, e, czn, czm, czp, kd);
      quad_kappa<float>(G, k32, e, czn, czm, czp, kk);
      const float dg = diag6T<float>(kk);
      const double uc = un(c);
      double acc = diag6(kd) * uc;
      if (i > 1) acc = __fma_rn(-kd[0], un(c - 1), acc);
      if (i < n) acc = __fma_rn(-kd[1], un(c + 1), acc);
      if (j > 1) acc = __fma_rn(-kd[2], un(c - n), acc);
      if (j < n) acc = __fma_rn(-kd[3], un(c + n), acc);
      if (k > 1) acc = __fma_rn(-kd[4], un(c - n2), acc);
      if (k < n) acc = __fma_rn(-kd[5], un(c + n2), acc);
      if (upd != 0.0) Ud[c] = uc;
      const double f = fval(P, S, i, j, k);
      const double rv = f - acc;
      const float r32 = (float)(rv * scale);
      R[c] = r32;
      cr_add_prod(arr, rv, rv);
      if (first) cr_add_prod(aff, f, f);
      g0 = __fma_rn((double)r32, (double)r32, g0);
      if (prec) g1 = __fma_rn((double)r32, (double)(r32 / dg), g1);
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    g0 += __shfl_xor(g0, m, 64);
    g1 += __shfl_xor(g1, m, 64);
  }
  if (lane == 0) {
    redd[w][0] = g0;
    redd[w][1] = g1;
  }
  IrPart* out = part + item;
  CrAcc a = cr_block_reduce(arr, redc);
  if (threadIdx.x == 0) out->rr = a;
  if (first) {
    a = cr_block_reduce(aff, redc);
    if (threadIdx.x == 0) out->ff = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out->g[0] = redd[0][0] + redd[1][0] + redd[2][0] + redd[3][0];
    out->g[1] = redd[0][1] + redd[1][1] + redd[2][1] + redd[3][1];
  }
}

// inner FP32 iteration sweeps (fast.hpp); p alternates by the parity of k_total
template <bool VEC, int OP>
__global__ __launch_bounds__(256) void k_fast32(const int2* __restrict__ items, int per, int nitems,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const IrState* __restrict__ st, const float* __restrict__ kap,
                                                float* __restrict__ d, float* __restrict__ r, float* __restrict__ p0,
                                                float* __restrict__ p1, IrPart* __restrict__ part, int ktab) {
  extern __shared__ double smem_raw[];
  float* smem = reinterpret_cast<float*>(smem_raw);
  __shared__ double red[4][2];
  const int item = item_of(blockIdx.x, per);
  if (item >= nitems) return;
  const int2 it = items[item];
  const int b = it.x;
  const IrState& s = st[b];
  if (s.mode != MODE_ITER) return;
  if (OP == FOP_UP2 && s.skip2) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const int ntab = P.g.ndir * P.g.nclass;
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) smem[e] = kap[S.kap_off + e];
  __syncthreads();
  QuadGeo G;
  quad_geo(G, P, it.y);
  const int par = s.k_total & 1;
  const float* Pold = (par ? p1 : p0) + S.off;
  float* Pn = (par ? p0 : p1) + S.off;
  DotAcc<float> a0, a1;
  a0.zero();
  a1.zero();
  fast_body<float, VEC, OP>(G, P.g, smem, smem + ktab, r + S.off, r + S.off, Pold, Pn, d + S.off,
                            (float)s.alpha, (float)s.beta, s.restart, s.prec, s.k_in == 0, a0, a1);
  double g0 = a0.a, g1 = a1.a;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    g0 += __shfl_xor(g0, m, 64);
    g1 += __shfl_xor(g1, m, 64);
  }
  if (lane == 0) {
    red[w][0] = g0;
    red[w][1] = g1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    IrPart* out = part + item;
    out->g[0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    out->g[1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
  }
}

__device__ __forceinline__ void ir_done(IrState& s, int status, int* active) {
  s.status = status;
  s.mode = MODE_DONE;
  s.t_done = wall_clock64();
  atomicSub(active, 1);
}

// end of an inner solve: schedule the outer update with the correction found
__device__ __forceinline__ void ir_end_inner(IrState& s, double rr_in) {
  s.upd = s.k_in > 0 ? 1.0 / s.scale : 0.0;
  double rho = (s.bb > 0.0 && rr_in >= 0.0) ? sqrt(rr_in / s.bb) : 1.0;
  if (!(rho <= 1.0)) rho = 1.0;
  if (rho < 0x1p-60) rho = 0x1p-60;
  s.scale = ldexp(s.scale, -ilogb(rho));
  s.mode = MODE_RESID;
}

__global__ __launch_bounds__(256) void k_ir_fin1(const SolveDev* __restrict__ sd, IrState* st,
                                                 const IrPart* __restrict__ part, int* active) {
  __shared__ double red[4][3];
  __shared__ CrAcc redc[4];
  const int b = blockIdx.x;
  const int mode = st[b].mode;
  if (mode == MODE_DONE) return;
  const SolveDev S = sd[b];
  IrState s = st[b];
  double g0 = 0.0, g1 = 0.0;
  CrAcc arr = cr_zero(), aff = cr_zero();
  for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) {
    const IrPart& q = part[S.item0 + t];
    g0 += q.g[0];
    g1 += q.g[1];
    if (mode == MODE_RESID) {
      arr = cr_combine(arr, q.rr);
      if (s.first) aff = cr_combine(aff, q.ff);
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int m = 32; m >= 1; m >>= 1) {
    g0 += __shfl_xor(g0, m, 64);
    g1 += __shfl_xor(g1, m, 64);
  }
  if (lane == 0) {
    red[w][0] = g0;
    red[w][1] = g1;
  }
  if (mode == MODE_RESID) {
    arr = cr_block_reduce(arr, redc);
    if (s.first) {
      CrAcc t = cr_block_reduce(aff, redc);
      if (threadIdx.x == 0) aff = t;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  g0 = g1 = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); q++) {
    g0 += red[q][0];
    g1 += red[q][1];
  }
  if (mode == MODE_ITER) {
    const double gam = g0;
    if (!(gam > 0.0) || !__builtin_isfinite(gam)) ir_end_inner(s, s.k_in > 0 ? s.rho : s.bb);
    else s.alpha = (double)(float)(s.rho / gam);
    st[b] = s;
    return;
  }
  // outer pass finished
  double rr, ff = s.ff;
  if (!cr_finalize(arr, &rr)) rr = arr.s + arr.lo;
  if (s.first) {
    if (!cr_finalize(aff, &ff)) ff = aff.s + aff.lo;
    s.ff = ff;
    s.thr = s.tol2 * ff;
    s.init_rr = rr;
    s.first = 0;
  }
  if (s.upd != 0.0) s.cur = 1 - s.cur;
  s.upd = 0.0;
  s.rr = rr;
  if (!__builtin_isfinite(rr)) ir_done(s, RBWS_SOLVE_NAN, active);
  else if (rr <= s.thr) ir_done(s, RBWS_SOLVE_CONVERGED, active);
  else if (s.outer >= s.max_outer) ir_done(s, RBWS_SOLVE_MAXITER, active);
  else {
    s.outer += 1;
    s.mode = MODE_ITER;
    s.k_in = 0;
    s.restart = 1;
    s.skip2 = 1;
    s.bb = g0;
    s.thr_in = s.eta2 * g0;
    s.rho = s.prec ? g1 : g0;
  }
  st[b] = s;
}

__global__ __launch_bounds__(256) void k_ir_fin2(const SolveDev* __restrict__ sd, IrState* st,
                                                 const IrPart* __restrict__ part) {
  __shared__ double red[4][2];
  const int b = blockIdx.x;
  if (st[b].mode != MODE_ITER) return;
  IrState s = st[b];
  if (s.skip2) {
    if (threadIdx.x == 0) st[b].skip2 = 0;
    return;
  }
  const SolveDev S = sd[b];
  double g0 = 0.0, g1 = 0.0;
  for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) {
    g0 += part[S.item0 + t].g[0];
    g1 += part[S.item0 + t].g[1];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int m = 32; m >= 1; m >>= 1) {
    g0 += __shfl_xor(g0, m, 64);
    g1 += __shfl_xor(g1, m, 64);
  }
  if (lane == 0) {
    red[w][0] = g0;
    red[w][1] = g1;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  g0 = g1 = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); q++) {
    g0 += red[q][0];
    g1 += red[q][1];
  }
  const double rr = g0, rs = s.prec ? g1 : g0;
  s.k_in += 1;
  s.k_total += 1;
  if (!__builtin_isfinite(rr) || rr <= s.thr_in || s.k_in >= s.inner_max) {
    ir_end_inner(s, rr);
  } else {
    s.beta = (double)(float)(rs / s.rho);
    s.rho = rs;
    s.restart = 0;
  }
  st[b] = s;
}

void ir_run(Batch& B, const IrOpts& o, hipStream_t s, std::vector<IrHost>& out) {
  RBWS_HIP(hipSetDevice(B.device));
  const int ns = B.nsolve;
  out.assign(ns, IrHost{});
  if (ns == 0) return;
  std::vector<IrState> init(ns);
  for (int b = 0; b < ns; b++) {
    IrState& c = init[b];
    std::memset(&c, 0, sizeof c);
    const double h2 = B.pd_h[B.sd_h[b].prob].h2;
    c.tol2 = o.tol * o.tol;
    c.eta2 = o.eta * o.eta;
    c.scale = ldexp(1.0, -ilogb(h2));
    c.mode = MODE_RESID;
    c.first = 1;
    c.status = -1;
    c.inner_max = o.inner_max;
    c.max_outer = o.max_outer;
    c.prec = o.prec;
  }
  IrState* st = (IrState*)B.state.get(sizeof(IrState) * ns, B.device);
  RBWS_HIP(hipMemcpyAsync(st, init.data(), sizeof(IrState) * ns, hipMemcpyHostToDevice, s));
  int* active = (int*)B.active.get(sizeof(int), B.device);
  RBWS_HIP(hipMemcpyAsync(active, &ns, sizeof(int), hipMemcpyHostToDevice, s));
  IrPart* part = (IrPart*)B.part.get(sizeof(IrPart) * B.nitems, B.device);
  double* u0 = (double*)B.x.ptr;
  RBWS_REQUIRE(u0 != nullptr && B.x.bytes >= sizeof(double) * B.total, RBWS_ESTATE, "initial guess missing");
  double* u1 = (double*)B.r.get(sizeof(double) * B.total, B.device);
  float* d = (float*)B.d32.get(sizeof(float) * B.total, B.device);
  float* r = (float*)B.r32.get(sizeof(float) * B.total, B.device);
  float* p = (float*)B.p32.get(sizeof(float) * B.total, B.device);
  float* p1 = (float*)B.p32b.get(sizeof(float) * B.total, B.device);
  const int2* items = (const int2*)B.items.ptr;
  const SolveDev* sd = (const SolveDev*)B.sd.ptr;
  const ProbDev* pd = (const ProbDev*)B.pd.ptr;
  const double* k64 = (const double*)B.kap64.ptr;
  const float* k32 = (const float*)B.kap32.ptr;
  const int ktab = (B.kap_max + 3) & ~3;
  const size_t lds_outer = (sizeof(double) + sizeof(float)) * ktab;
  const size_t lds_fast = sizeof(float) * (ktab + 2 * QPLANE);
  const int per = B.per, ni = B.nitems;
  const unsigned grid = grid_of(B);
  auto ap = B.vec ? k_fast32<true, FOP_AP> : k_fast32<false, FOP_AP>;
  auto up = B.vec ? k_fast32<true, FOP_UP2> : k_fast32<false, FOP_UP2>;
  const int check = o.check_every > 0 ? o.check_every : 8;
  const long long max_rounds = (long long)(o.inner_max + 2) * (o.max_outer + 1) + 16;
  for (long long round = 0; round < max_rounds; round++) {
    hipLaunchKernelGGL(ap, dim3(grid), dim3(256), lds_fast, s, items, per, ni, sd, pd, st, k32, d, r, p, p1, part, ktab);
    hipLaunchKernelGGL(k_ir_outer, dim3(grid), dim3(256), lds_outer, s, items, per, ni, sd, pd, st, k64, k32, u0,
                       u1, d, r, part, ktab);
    hipLaunchKernelGGL(k_ir_fin1, dim3(ns), dim3(256), 0, s, sd, st, (const IrPart*)part, active);
    hipLaunchKernelGGL(up, dim3(grid), dim3(256), lds_fast, s, items, per, ni, sd, pd, st, k32, d, r, p, p1, part, ktab);
    hipLaunchKernelGGL(k_ir_fin2, dim3(ns), dim3(256), 0, s, sd, st, (const IrPart*)part);
    RBWS_HIP(hipGetLastError());
    if ((round + 1) % check == 0) {
      RBWS_HIP(hipMemcpyAsync(B.active_host, active, sizeof(int), hipMemcpyDeviceToHost, s));
      RBWS_HIP(hipStreamSynchronize(s));
      if (*B.active_host == 0) break;
    }
  }
  std::vector<IrState> h(ns);
  RBWS_HIP(hipMemcpyAsync(h.data(), st, sizeof(IrState) * ns, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < ns; b++) {
    IrHost& q = out[b];
    q.iters = h[b].k_total;
    q.outer = h[b].outer;
    q.status = h[b].status < 0 ? RBWS_SOLVE_MAXITER : h[b].status;
    q.cur = h[b].cur;
    q.init_rr = h[b].init_rr;
    q.rr = h[b].rr;
    q.ff = h[b].ff;
    q.t_done = h[b].t_done;
  }
}

}  // namespace rbws
