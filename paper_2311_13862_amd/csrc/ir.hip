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
#include <cstdlib>
#include <cstring>

#include "fast.hpp"
#include "mg.hpp"

namespace rbws {

// Outer pass (FP64) of every solve whose mode is RESID (fast.hpp, outer_body).
// SRC: some problem of the batch has a parameter-dependent source; without it
// f_h is the constant h^2 and the exponential's code stays out of the kernel
// (it would otherwise size the register allocation of the f = 1 case too).
template <bool VEC, bool SRC>
__device__ __forceinline__ void k_ir_outer_item(int item, const int2* __restrict__ items,
                                                  const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                  const IrState* __restrict__ st, const double* __restrict__ kap64,
                                                  const float* __restrict__ kap32, double* __restrict__ u0,
                                                  double* __restrict__ u1, const float* __restrict__ d,
                                                  float* __restrict__ r, IrPart* __restrict__ part,
                                                  double* __restrict__ fc, int ktab) {
  extern __shared__ __align__(16) double lds[];
  __shared__ double redd[4][2];
  __shared__ CrAcc redc[4];
  __shared__ int zk[kZkLen];
  __syncthreads();  // LDS of the previous item is free
  const int2 it = items[item];
  const int b = it.x;
  if (st[b].mode != MODE_RESID) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const GridDev& g = P.g;
  const int ntab = g.ndir * g.nclass;
  double* k64 = lds;
  float* k32 = reinterpret_cast<float*>(lds + ktab);
  double* plane = lds + ktab + (ktab + 1) / 2;
  QuadGeo G;
  quad_geo(G, P, it.y);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) {
    k32[e] = kap32[S.kap_off + e];
    k64[e] = kap64[S.kap_off + e];
  }
  zk_stage(zk, g, G);
  __syncthreads();
  const IrState& s = st[b];
  const int first = s.first;
  double g0 = 0.0, g1 = 0.0;
  CrAcc arr = cr_zero(), aff = cr_zero();
  // a parameter-dependent source is evaluated (exponential rounded to nearest)
  // on the solve's first outer pass and kept in fc for the later ones
  double* F = (SRC && fc != nullptr && P.f_kind != RBWS_F_ONE) ? fc + S.off : nullptr;
  const double h2 = P.h2;
  auto fv = [&](int i, int j, int k) -> double {
    if constexpr (!SRC) {
      return h2;
    } else {
      if (F == nullptr) return fval(P, S, i, j, k);
      const long long c = vidx(g.n, i, j, k);
      if (!first) return F[c];
      const double v = fval(P, S, i, j, k);
      F[c] = v;
      return v;
    }
  };
  outer_body<VEC>(G, g, k64, k32, plane, (s.cur ? u1 : u0) + S.off, (s.cur ? u0 : u1) + S.off, d + S.off,
                  r + S.off, s.upd, s.scale, s.prec, first, fv, arr, aff, g0, g1);
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

// With a parameter-dependent source: three waves per SIMD, 167 VGPRs without
// spills (177 and two waves unbounded).  With f = 1: four waves, 128 VGPRs, the
// few spilled values stored and reloaded outside the z-loop (0.95 against
// 1.01-1.05 ms per launch at 1024 x 128^3, where three waves took 0.95-0.98).
template <bool VEC, bool SRC>
__global__ __launch_bounds__(256, SRC ? 3 : 4) void k_ir_outer(const int2* __restrict__ items, const int* __restrict__ list,
                                                  const int* __restrict__ cnt, int nitems,
                                                  const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                  const IrState* __restrict__ st, const double* __restrict__ kap64,
                                                  const float* __restrict__ kap32, double* __restrict__ u0,
                                                  double* __restrict__ u1, const float* __restrict__ d,
                                                  float* __restrict__ r, IrPart* __restrict__ part,
                                                  double* __restrict__ fc, int ktab) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step)
    k_ir_outer_item<VEC, SRC>(list ? list[w] : w, items, sd, pd, st, kap64, kap32, u0, u1, d, r, part, fc, ktab);
}

// inner FP32 iteration sweeps (fast.hpp); p alternates by the parity of k_total
template <bool VEC, int OP, bool CACHED>
__device__ __forceinline__ void k_fast32_item(int item, const int2* __restrict__ items,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const IrState* __restrict__ st, const float* __restrict__ kap,
                                                float* __restrict__ d, float* __restrict__ r, float* __restrict__ p0,
                                                float* __restrict__ p1, IrPart* __restrict__ part, int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  float* smem = reinterpret_cast<float*>(smem_raw);
  __shared__ double red[4][2];
  __shared__ int zk[kZkLen];
  __syncthreads();  // LDS of the previous item is free
  const int2 it = items[item];
  const int b = it.x;
  const IrState& s = st[b];
  if (s.mode != MODE_ITER) return;
  if (OP == FOP_UP2 && s.skip2) return;
  const SolveDev S = sd[b];
  const ProbDev& P = pd[S.prob];
  const int ntab = P.g.ndir * P.g.nclass;
  QuadGeo G;
  quad_geo(G, P, it.y);
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) smem[e] = kap[S.kap_off + e];
  zk_stage(zk, P.g, G);
  __syncthreads();
  const int par = s.k_total & 1;
  const float* Pold = (par ? p1 : p0) + S.off;
  float* Pn = (par ? p0 : p1) + S.off;
  double g0 = 0.0, g1 = 0.0;
  if (CACHED) {
    fast_body32<VEC, OP>(G, P.g, smem, smem + ktab, r + S.off, r + S.off, Pold, Pn, d + S.off,
                         (float)s.alpha, (float)s.beta, s.restart, s.prec, s.k_in == 0, g0, g1);
  } else {
    DotAcc<float> a0, a1;
    a0.zero();
    a1.zero();
    fast_body<float, VEC, OP>(G, P.g, smem, smem + ktab, r + S.off, r + S.off, Pold, Pn, d + S.off,
                              (float)s.alpha, (float)s.beta, s.restart, s.prec, s.k_in == 0, a0, a1);
    g0 = a0.a;
    g1 = a1.a;
  }
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

template <bool VEC, int OP, bool CACHED>
__global__ __launch_bounds__(256) void k_fast32(const int2* __restrict__ items, const int* __restrict__ list,
                                                const int* __restrict__ cnt, int nitems,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const IrState* __restrict__ st, const float* __restrict__ kap,
                                                float* __restrict__ d, float* __restrict__ r,
                                                float* __restrict__ p0, float* __restrict__ p1,
                                                IrPart* __restrict__ part, int ktab) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step)
    k_fast32_item<VEC, OP, CACHED>(list ? list[w] : w, items, sd, pd, st, kap, d, r, p0, p1, part, ktab);
}

__device__ __forceinline__ void ir_done(IrState& s, int status, int* active) {
  s.status = status;
  s.mode = MODE_DONE;
  s.t_done = wall_clock64();
  atomicSub(active, 1);
}

// end of an inner solve: schedule the outer update with the correction found
// (with reliable updates the next outer step keeps the direction p, rescaled)
__device__ __forceinline__ void ir_end_inner(IrState& s, double rr_in, int dir_ok) {
  s.upd = s.k_in > 0 ? 1.0 / s.scale : 0.0;
  double rho = (s.bb > 0.0 && rr_in >= 0.0) ? sqrt(rr_in / s.bb) : 1.0;
  if (!(rho <= 1.0)) rho = 1.0;
  if (rho < 0x1p-60) rho = 0x1p-60;
  const double ns = ldexp(s.scale, -ilogb(rho));
  s.rescale = ns / s.scale;
  s.scale = ns;
  s.dir_ok = dir_ok && s.k_in > 0;
  s.mode = MODE_RESID;
}

__global__ __launch_bounds__(256) void k_ir_fin1(const SolveDev* __restrict__ sd, IrState* st,
                                                 const IrPart* __restrict__ part, int* active, Lists L) {
  __shared__ double red[4][3];
  __shared__ CrAcc redc[4];
  __shared__ int flag, slot;
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) {  // the ap and res sweeps and the last V-cycle are done
    L.cnt[WL_AP] = 0;
    L.cnt[WL_RES] = 0;
    for (int q = 0; q < WL_MAXPROB; q++) L.cnt[WL_MG + q] = 0;
  }
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
  if (threadIdx.x == 0) {
    g0 = g1 = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) {
      g0 += red[q][0];
      g1 += red[q][1];
    }
    if (mode == MODE_ITER) {
      const double gam = g0;
      if (!(gam > 0.0) || !__builtin_isfinite(gam)) ir_end_inner(s, s.k_in > 0 ? s.rho : s.bb, 0);
      else s.alpha = (double)(float)(s.rho / gam);
    } else {
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
        const double rho_new = s.prec ? g1 : g0;
        s.outer += 1;
        s.mode = MODE_ITER;
        s.k_in = 0;
        s.skip2 = 1;
        s.bb = g0;
        // reduce by eta, and at least to eta ||f|| (scaled units): a start whose
        // residual exceeds ||f|| needs no more outer steps than the zero start
        s.thr_in = s.eta2 * fmin(g0, s.ff * s.scale * s.scale);
        if (s.mg) {
          // beta, restart and rho follow the V-cycle on the new right-hand side (k_ir_fin_mg)
        } else if (s.reliable && s.dir_ok && s.rho > 0.0) {
          // continue CG with the true residual: p <- s + beta p, p rescaled by s.rescale
          s.beta = (double)(float)(rho_new / (s.rescale * s.rho));
          s.restart = 0;
        } else {
          s.restart = 1;
        }
        if (!s.mg) s.rho = rho_new;
      }
    }
    st[b] = s;
    flag = s.mode == MODE_ITER && !s.skip2;
  }
  __syncthreads();
  if (flag) list_push(L.up, L.cnt + WL_UP, S.item0, S.ntiles, &slot);
}

__global__ __launch_bounds__(256) void k_ir_fin2(const SolveDev* __restrict__ sd, IrState* st,
                                                 const IrPart* __restrict__ part, Lists L, int* need) {
  __shared__ double red[4][2];
  __shared__ int flag, slot;
  const int b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) L.cnt[WL_UP] = 0;  // the up sweep of this round is done
  const int mode = st[b].mode;
  if (need && threadIdx.x == 0) need[b] = 0;
  if (mode == MODE_DONE) return;
  const SolveDev S = sd[b];
  if (mode == MODE_RESID) {
    list_push(L.res, L.cnt + WL_RES, S.item0, S.ntiles, &slot);
    return;
  }
  IrState s = st[b];
  if (s.skip2) {
    if (threadIdx.x == 0) {
      st[b].skip2 = 0;
      if (need) {  // the V-cycle on the new right-hand side
        need[b] = 1;
        st[b].nvc += 1;
        const int q = sd[b].prob;
        L.mg[L.cnt[WL_SEG + q] + atomicAdd(&L.cnt[WL_MG + q], 1)] = L.gidx[b];
      }
    }
    list_push(L.ap, L.cnt + WL_AP, S.item0, S.ntiles, &slot);
    return;
  }
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
  if (threadIdx.x == 0) {
    g0 = g1 = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) {
      g0 += red[q][0];
      g1 += red[q][1];
    }
    const double rr = g0, rs = s.prec ? g1 : g0;
    s.k_in += 1;
    s.k_total += 1;
    if (!__builtin_isfinite(rr) || rr <= s.thr_in || s.k_in >= s.inner_max) {
      ir_end_inner(s, rr, __builtin_isfinite(rr) ? 1 : 0);
    } else if (s.mg) {
      s.restart = 0;  // beta and rho follow the V-cycle (k_ir_fin_mg)
      s.nvc += 1;
      need[b] = 1;
      L.mg[L.cnt[WL_SEG + S.prob] + atomicAdd(&L.cnt[WL_MG + S.prob], 1)] = L.gidx[b];
    } else {
      s.beta = (double)(float)(rs / s.rho);
      s.rho = rs;
      s.restart = 0;
    }
    st[b] = s;
    flag = s.mode;
  }
  __syncthreads();
  if (flag == MODE_ITER) list_push(L.ap, L.cnt + WL_AP, S.item0, S.ntiles, &slot);
  else list_push(L.res, L.cnt + WL_RES, S.item0, S.ntiles, &slot);
}

// r^T s of the inner solve (FP32 vectors, FP64 accumulation) over listed tiles, into g[2]
__device__ __forceinline__ void k_dot_rs32_item(int item, const int2* __restrict__ items,
                                                const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                const float* __restrict__ r, const float* __restrict__ sv,
                                                IrPart* __restrict__ part) {
  __shared__ double red[4];
  __syncthreads();
  const int2 it = items[item];
  const SolveDev S = sd[it.x];
  const ProbDev& P = pd[S.prob];
  QuadGeo G;
  quad_geo(G, P, it.y);
  const int n = P.g.n;
  double a = 0.0;
  for (int k = G.kb; k <= G.ke; k++) {
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (e >= G.nv) continue;
      const long long c = S.off + vidx(n, G.i + e, G.j, k);
      a = __fma_rn((double)r[c], (double)sv[c], a);
    }
  }
  for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[item].g[2] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_dot_rs32(const int2* __restrict__ items, const int* __restrict__ list,
                                                  const int* __restrict__ cnt, int nitems,
                                                  const SolveDev* __restrict__ sd, const ProbDev* __restrict__ pd,
                                                  const float* __restrict__ r, const float* __restrict__ sv,
                                                  IrPart* __restrict__ part) {
  const WorkRange R = work_range(cnt ? *cnt : nitems);
  for (int w = R.w; w < R.w1; w += R.step) k_dot_rs32_item(list ? list[w] : w, items, sd, pd, r, sv, part);
}

// after the V-cycle: rho' = r^T s; beta = rho' / rho, or after an outer step the
// reliable-update continuation beta = rho' / (rescale rho) (or a restart)
__global__ __launch_bounds__(256) void k_ir_fin_mg(const SolveDev* __restrict__ sd, IrState* st,
                                                   const IrPart* __restrict__ part, const int* __restrict__ need) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  if (!need[b]) return;
  const SolveDev S = sd[b];
  double g = 0.0;
  for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) g += part[S.item0 + t].g[2];
  for (int m = 32; m >= 1; m >>= 1) g += __shfl_xor(g, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x != 0) return;
  g = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); q++) g += red[q];
  IrState s = st[b];
  if (s.k_in == 0) {
    if (s.reliable && s.dir_ok && s.rho > 0.0) {
      s.beta = (double)(float)(g / (s.rescale * s.rho));
      s.restart = 0;
    } else {
      s.restart = 1;
    }
  } else {
    s.beta = (double)(float)(g / s.rho);
  }
  s.rho = g;
  st[b] = s;
}

// bit 0: A.p sweep with register-cached coefficients; bit 1: the same for the
// update sweep.  RBWS_SWEEP32 overrides the default (for tuning runs).  The
// default 2 measured fastest on whole-row 128 x 8 tiles at 128^3: the A.p sweep
// reads the class table (80 VGPRs, six waves per SIMD), the update sweep keeps
// its coefficients in registers.
static int g_sweep32 = -1;
int sweep32_variant() {
  if (g_sweep32 < 0) {
    const char* e = std::getenv("RBWS_SWEEP32");
    g_sweep32 = e ? std::atoi(e) & 3 : 2;
  }
  return g_sweep32;
}
void set_sweep32_variant(int v) { g_sweep32 = v & 3; }

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
    c.reliable = o.reliable;
    c.rescale = 1.0;
    if (o.prec == RBWS_PREC_MG) {
      c.prec = 0;  // the sweeps form ||r||^2 only; s and r^T s come from the V-cycle
      c.mg = 1;
    }
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
  // f_h of the solves with a parameter-dependent source, formed on each
  // solve's first outer pass (its exponentials cost more than the pass's
  // other arithmetic) and read by the later passes
  bool gauss = false;
  for (const Problem* P : B.probs) gauss = gauss || P->desc.f_kind != RBWS_F_ONE;
  double* fcache = gauss ? (double*)B.fc.get(sizeof(double) * B.total, B.device) : nullptr;
  float* p = (float*)B.p32.get(sizeof(float) * B.total, B.device);
  float* p1 = (float*)B.p32b.get(sizeof(float) * B.total, B.device);
  const int2* items = (const int2*)B.items.ptr;
  const SolveDev* sd = (const SolveDev*)B.sd.ptr;
  const ProbDev* pd = (const ProbDev*)B.pd.ptr;
  const double* k64 = (const double*)B.kap64.ptr;
  const float* k32 = (const float*)B.kap32.ptr;
  const int ktab = (B.kap_max + 3) & ~3;
  const size_t lds_outer = sizeof(double) * (ktab + (ktab + 1) / 2 + 2 * QPLANE);
  auto outer = B.vec ? (gauss ? k_ir_outer<true, true> : k_ir_outer<true, false>)
                     : (gauss ? k_ir_outer<false, true> : k_ir_outer<false, false>);
  const size_t lds_fast = sizeof(float) * (ktab + 2 * QPLANE);
  const int ni = B.nitems;
  // sweep variants: coefficients cached in registers or looked up per plane
  const int var = sweep32_variant();
  auto ap = (var & 1) ? (B.vec ? k_fast32<true, FOP_AP, true> : k_fast32<false, FOP_AP, true>)
                      : (B.vec ? k_fast32<true, FOP_AP, false> : k_fast32<false, FOP_AP, false>);
  auto up = (var & 2) ? (B.vec ? k_fast32<true, FOP_UP2, true> : k_fast32<false, FOP_UP2, true>)
                      : (B.vec ? k_fast32<true, FOP_UP2, false> : k_fast32<false, FOP_UP2, false>);
  const unsigned g_ap = persistent_grid((const void*)ap, lds_fast, ni, B.device);
  const unsigned g_up = persistent_grid((const void*)up, lds_fast, ni, B.device);
  const unsigned g_res = persistent_grid((const void*)outer, lds_outer, ni, B.device);
  const Lists L = lists_init(B, s);
  const bool mg = o.prec == RBWS_PREC_MG;
  MgRun* mgr = nullptr;
  float* sv = r;  // the vector the direction update reads: r (P = I, Jacobi in-kernel) or s
  int* need = nullptr;
  if (mg) {
    mgr = mg_prepare(B, o.mg_nu, o.mg_omega, true, s);
    sv = (float*)B.sv32.get(sizeof(float) * B.total, B.device);
    need = (int*)B.need.get(sizeof(int) * ns, B.device);
    std::vector<int> z(ns, 0);
    RBWS_HIP(hipMemcpyAsync(need, z.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    RBWS_HIP(hipStreamSynchronize(s));
  }
  const unsigned g_dot = mg ? persistent_grid((const void*)k_dot_rs32, 0, ni, B.device) : 0;
  const int check = o.check_every > 0 ? o.check_every : 8;
  const long long max_rounds = (long long)(o.inner_max + 2) * (o.max_outer + 1) + 16;
  KernelTimer& kt = ktimer();
  const bool graph = !(o.flags & RBWS_FLAG_NO_GRAPH) && !kt.on;
  run_rounds(B, active, max_rounds, check, graph, s, [&](hipStream_t q) {
    kt.begin(q, KK_AP);
    hipLaunchKernelGGL(ap, dim3(g_ap), dim3(256), lds_fast, q, items, L.ap, L.cnt + WL_AP, ni, sd, pd, st, k32, d,
                       sv, p, p1, part, ktab);
    kt.end(q);
    kt.begin(q, KK_RESID);
    hipLaunchKernelGGL(outer, dim3(g_res), dim3(256), lds_outer, q, items, L.res, L.cnt + WL_RES, ni, sd, pd, st,
                       k64, k32, u0, u1, d, r, part, fcache, ktab);
    kt.end(q);
    kt.begin(q, KK_FIN1);
    hipLaunchKernelGGL(k_ir_fin1, dim3(ns), dim3(256), 0, q, sd, st, (const IrPart*)part, active, L);
    kt.end(q);
    kt.begin(q, KK_UP2);
    hipLaunchKernelGGL(up, dim3(g_up), dim3(256), lds_fast, q, items, L.up, L.cnt + WL_UP, ni, sd, pd, st, k32, d,
                       r, p, p1, part, ktab);
    kt.end(q);
    kt.begin(q, KK_FIN2);
    hipLaunchKernelGGL(k_ir_fin2, dim3(ns), dim3(256), 0, q, sd, st, (const IrPart*)part, L, need);
    kt.end(q);
    if (mg) {
      const bool fused = mg_apply(mgr, B, r, sv, L, part, q);  // times its own kernels
      kt.begin(q, KK_MG);
      if (!fused)
        hipLaunchKernelGGL(k_dot_rs32, dim3(g_dot), dim3(256), 0, q, items, (const int*)L.ap,
                           (const int*)(L.cnt + WL_AP), ni, sd, pd, (const float*)r, (const float*)sv, part);
      hipLaunchKernelGGL(k_ir_fin_mg, dim3(ns), dim3(256), 0, q, sd, st, (const IrPart*)part, (const int*)need);
      kt.end(q);
    }
  });
  std::vector<IrState> h(ns);
  RBWS_HIP(hipMemcpyAsync(h.data(), st, sizeof(IrState) * ns, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < ns; b++) {
    IrHost& q = out[b];
    q.iters = h[b].k_total;
    q.outer = h[b].outer;
    q.status = h[b].status < 0 ? RBWS_SOLVE_MAXITER : h[b].status;
    q.cur = h[b].cur;
    q.nvc = h[b].nvc;
    q.init_rr = h[b].init_rr;
    q.rr = h[b].rr;
    q.ff = h[b].ff;
    q.t_done = h[b].t_done;
  }
}

}  // namespace rbws
