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

#include "stencil.hpp"

namespace rbws {

struct IrState {
  double thr, ff, tol2, rr, init_rr, scale, upd, eta2;
  double rho, alpha, beta, thr_in, bb;
  int outer, mode, first, status, cur, k_in, k_total, restart, skip2, inner_max, max_outer, prec;
  unsigned long long t_done;
};

struct IrPart {
  CrAcc rr, ff;
  double g[3];
  double pad;
};

enum { IOP_PUP = 0, IOP_AP = 1, IOP_UP2 = 2 };

template <int OP>
__global__ __launch_bounds__(256) void k_ir_sweep(const int2* __restrict__ items, const SolveDev* __restrict__ sd,
                                                  const ProbDev* __restrict__ pd, const IrState* __restrict__ st,
                                                  const double* __restrict__ kap64, const float* __restrict__ kap32,
                                                  double* __restrict__ u0, double* __restrict__ u1,
                                                  float* __restrict__ d, float* __restrict__ r,
                                                  float* __restrict__ p, IrPart* __restrict__ part, int ntab_max) {
  extern __shared__ double lds[];
  __shared__ double redd[4][3];
  __shared__ CrAcc redc[4];
  const int2 it = items[blockIdx.x];
  const int b = it.x, tile = it.y;
  const int mode = st[b].mode;
  bool run;
  if (OP == IOP_PUP) run = mode == MODE_ITER;
  else if (OP == IOP_AP) run = mode == MODE_ITER || mode == MODE_RESID;
  else run = mode == MODE_ITER && st[b].skip2 == 0;
  if (!run) return;
  const bool outer = (OP == IOP_AP && mode == MODE_RESID);
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const GridDev& g = P.g;
  const int ntab = g.ndir * g.nclass;
  double* k64 = lds;
  float* k32 = reinterpret_cast<float*>(lds + ntab_max);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) {
    k32[e] = kap32[S.kap_off + e];
    if (outer) k64[e] = kap64[S.kap_off + e];
  }
  __syncthreads();
  const int n = g.n;
  const long long n2 = (long long)n * n;
  const int tx = tile % P.ntx, ty = (tile / P.ntx) % P.nty, tz = tile / (P.ntx * P.nty);
  const int i = tx * P.TX + (int)threadIdx.x % P.TX + 1, j = ty * P.TY + (int)threadIdx.x / P.TX + 1;
  const bool act = i <= n && j <= n;
  const int kb = tz * P.TZ + 1, ke = min(n, (tz + 1) * P.TZ);
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  const int oY = g.ndir == 3 ? g.nclass : 0, oZ = g.ndir == 3 ? 2 * g.nclass : 0;
  const IrState& s = st[b];
  const int prec = s.prec;
  const float alpha = (float)s.alpha, beta = (float)s.beta;
  const int restart = s.restart, first_inner = s.k_in == 0, first = s.first;
  const double upd = s.upd, scale = s.scale;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  CrAcc arr = cr_zero(), aff = cr_zero();
  if (act) {
    const int cxn = g.code[0][0][i - 1], cxm = g.code[0][1][i - 1], cxp = g.code[0][1][i];
    const int cyn = g.code[1][0][j - 1], cym = g.code[1][1][j - 1], cyp = g.code[1][1][j];
    const int bXm = (cxm * N1 + cyn) * N2, bXp = (cxp * N1 + cyn) * N2;
    const int bYm = oY + (cxn * N1 + cym) * N2, bYp = oY + (cxn * N1 + cyp) * N2;
    const int bZ = oZ + (cxn * N1 + cyn) * N2;
    float* D = d + S.off;
    float* R = r + S.off;
    float* Pv = p + S.off;
    const double* Us = (s.cur ? u1 : u0) + S.off;
    double* Ud = (s.cur ? u0 : u1) + S.off;
    for (int k = kb; k <= ke; k++) {
      const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
      const int ix[6] = {bXm + czn, bXp + czn, bYm + czn, bYp + czn, bZ + czm, bZ + czp};
      const long long c = vidx(n, i, j, k);
      float kk[6];
#pragma unroll
      for (int t = 0; t < 6; t++) kk[t] = k32[ix[t]];
      const float dg = ((((kk[0] + kk[1]) + kk[2]) + kk[3]) + kk[4]) + kk[5];
      if (OP == IOP_PUP) {
        const float rv = R[c];
        const float sv = prec ? rv / dg : rv;
        Pv[c] = restart ? sv : fmaf(beta, Pv[c], sv);
      } else if (outer) {
        // u_new = u + upd d at the point and its neighbours, then r = f - A64 u_new
        double kd[6];
#pragma unroll
        for (int t = 0; t < 6; t++) kd[t] = k64[ix[t]];
        const double dgd = diag6(kd);
        auto un = [&](long long e) { return upd != 0.0 ? __fma_rn(upd, (double)D[e], Us[e]) : Us[e]; };
        const double uc = un(c);
        double acc = dgd * uc;
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
      } else {
        float q = dg * Pv[c];
        if (i > 1) q = fmaf(-kk[0], Pv[c - 1], q);
        if (i < n) q = fmaf(-kk[1], Pv[c + 1], q);
        if (j > 1) q = fmaf(-kk[2], Pv[c - n], q);
        if (j < n) q = fmaf(-kk[3], Pv[c + n], q);
        if (k > 1) q = fmaf(-kk[4], Pv[c - n2], q);
        if (k < n) q = fmaf(-kk[5], Pv[c + n2], q);
        if (OP == IOP_AP) {
          g0 = __fma_rn((double)Pv[c], (double)q, g0);
        } else {
          const float pv = Pv[c];
          D[c] = first_inner ? alpha * pv : fmaf(alpha, pv, D[c]);
          const float rv = fmaf(-alpha, q, R[c]);
          R[c] = rv;
          g0 = __fma_rn((double)rv, (double)rv, g0);
          if (prec) g1 = __fma_rn((double)rv, (double)(rv / dg), g1);
        }
      }
    }
  }
  if (OP == IOP_PUP) return;
  // block reduction of the plain FP64 sums (and the exact-path accumulators)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    g0 += __shfl_xor(g0, m, 64);
    g1 += __shfl_xor(g1, m, 64);
    g2 += __shfl_xor(g2, m, 64);
  }
  if (lane == 0) {
    redd[w][0] = g0;
    redd[w][1] = g1;
    redd[w][2] = g2;
  }
  IrPart* out = part + blockIdx.x;
  if (outer) {
    CrAcc a = cr_block_reduce(arr, redc);
    if (threadIdx.x == 0) out->rr = a;
    if (first) {
      a = cr_block_reduce(aff, redc);
      if (threadIdx.x == 0) out->ff = a;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 0; t < 3; t++) {
      double v = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); q++) v += redd[q][t];
      out->g[t] = v;
    }
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
  const int2* items = (const int2*)B.items.ptr;
  const SolveDev* sd = (const SolveDev*)B.sd.ptr;
  const ProbDev* pd = (const ProbDev*)B.pd.ptr;
  const double* k64 = (const double*)B.kap64.ptr;
  const float* k32 = (const float*)B.kap32.ptr;
  const size_t lds = (sizeof(double) + sizeof(float)) * B.kap_max;
  const int check = o.check_every > 0 ? o.check_every : 8;
  const long long max_rounds = (long long)(o.inner_max + 2) * (o.max_outer + 1) + 16;
  for (long long round = 0; round < max_rounds; round++) {
    hipLaunchKernelGGL(k_ir_sweep<IOP_PUP>, dim3(B.nitems), dim3(256), lds, s, items, sd, pd, st, k64, k32,
                       u0, u1, d, r, p, part, B.kap_max);
    hipLaunchKernelGGL(k_ir_sweep<IOP_AP>, dim3(B.nitems), dim3(256), lds, s, items, sd, pd, st, k64, k32,
                       u0, u1, d, r, p, part, B.kap_max);
    hipLaunchKernelGGL(k_ir_fin1, dim3(ns), dim3(256), 0, s, sd, st, (const IrPart*)part, active);
    hipLaunchKernelGGL(k_ir_sweep<IOP_UP2>, dim3(B.nitems), dim3(256), lds, s, items, sd, pd, st, k64, k32,
                       u0, u1, d, r, p, part, B.kap_max);
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
