// stencil.hpp -- device helpers shared by the FP64 and FP32 sweeps.
#pragma once
#include "solver.hpp"

namespace rbws {

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long vidx(int n, int i, int j, int k) {
  return ((long long)(k - 1) * n + (j - 1)) * n + (i - 1);
}

__device__ __forceinline__ double fval(const ProbDev& P, const SolveDev& S, int i, int j, int k) {
  if (P.f_kind == RBWS_F_ONE) return P.h2;
  double dx = i * P.h - S.x0[0], dy = j * P.h - S.x0[1], dz = k * P.h - S.x0[2];
  return P.h2 * exp(-(dx * dx + dy * dy + dz * dz) / P.gw);
}

// the six face coefficients of point (i,j,k) from a class table in any memory
__device__ __forceinline__ void point_kappa(const GridDev& g, const double* kap, int i, int j, int k,
                                            double kk[6]) {
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  const double* kX = kap;
  const double* kY = kap + (g.ndir == 3 ? g.nclass : 0);
  const double* kZ = kap + (g.ndir == 3 ? 2 * g.nclass : 0);
  int cxn = g.code[0][0][i - 1], cxm = g.code[0][1][i - 1], cxp = g.code[0][1][i];
  int cyn = g.code[1][0][j - 1], cym = g.code[1][1][j - 1], cyp = g.code[1][1][j];
  int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
  kk[0] = kX[(cxm * N1 + cyn) * N2 + czn];
  kk[1] = kX[(cxp * N1 + cyn) * N2 + czn];
  kk[2] = kY[(cxn * N1 + cym) * N2 + czn];
  kk[3] = kY[(cxn * N1 + cyp) * N2 + czn];
  kk[4] = kZ[(cxn * N1 + cyn) * N2 + czm];
  kk[5] = kZ[(cxn * N1 + cyn) * N2 + czp];
}

__device__ __forceinline__ double diag6(const double kk[6]) {
  return ((((kk[0] + kk[1]) + kk[2]) + kk[3]) + kk[4]) + kk[5];
}

// (A v)_c in the fixed order: d v_c, then fma with interior neighbours x-,x+,y-,y+,z-,z+
__device__ __forceinline__ double stencil(const double kk[6], double dg, const double* v, long long c,
                                          int n, int i, int j, int k) {
  const long long n2 = (long long)n * n;
  double acc = dg * v[c];
  if (i > 1) acc = __fma_rn(-kk[0], v[c - 1], acc);
  if (i < n) acc = __fma_rn(-kk[1], v[c + 1], acc);
  if (j > 1) acc = __fma_rn(-kk[2], v[c - n], acc);
  if (j < n) acc = __fma_rn(-kk[3], v[c + n], acc);
  if (k > 1) acc = __fma_rn(-kk[4], v[c - n2], acc);
  if (k < n) acc = __fma_rn(-kk[5], v[c + n2], acc);
  return acc;
}

}  // namespace rbws
