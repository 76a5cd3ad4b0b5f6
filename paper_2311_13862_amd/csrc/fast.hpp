// fast.hpp -- the two bandwidth-bound sweeps of a Krylov iteration on gfx950.
//
// Tile: 32 x 32 grid columns, marching through a z-range of the solve.  A
// thread owns 4 consecutive x points of one row (vector loads); the values of
// the current plane sit in a double-buffered LDS plane with a one-point halo,
// the planes below and above in registers.  Points outside the domain carry
// the value 0, which is exact here: fma(-kappa, +0, acc) == acc for every acc,
// so the result is bitwise that of skipping boundary neighbours.
//
//   AP  (iteration k): p_new = s + beta p_old (s = P(r); p_new = s on a
//       restart), written to the other p buffer; the halo values of p_new are
//       recomputed from r and p_old; gamma = p_new . A p_new.
//   UP2 (iteration k): q = A p_new; x += alpha p_new (FP32 refinement: the
//       correction d); r -= alpha q; ||r||^2 and r . P(r).
// p alternates between two buffers because a tile reads p_old at its halo
// while the neighbouring tile writes p_new there.
#pragma once
#include "stencil.hpp"

namespace rbws {

constexpr int QX = 32, QY = 32;                 // tile columns (x, y)
constexpr int QS = 36;                          // LDS row stride (elements)
constexpr int QROWS = QY + 2;                   // rows with the two halo rows
constexpr int QPLANE = QROWS * QS + 2 * QROWS;  // plane buffer: rows + left/right halo columns

// Blocks are dealt round-robin to the 8 XCDs; give every XCD a contiguous run
// of work items so that the tiles of one solve share one L2.
__device__ __forceinline__ int item_of(int bid, int per) { return (bid & 7) * per + (bid >> 3); }

template <typename T> struct V4T;
template <> struct V4T<float> { typedef float4 t; };
template <> struct V4T<double> { typedef double4 t; };

template <typename T, bool VEC>
__device__ __forceinline__ void ld4(const T* __restrict__ a, long long c, int nv, T v[4]) {
  if (VEC && nv == 4) {
    const typename V4T<T>::t q = *reinterpret_cast<const typename V4T<T>::t*>(a + c);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = e < nv ? a[c + e] : T(0);
  }
}

template <typename T, bool VEC>
__device__ __forceinline__ void st4(T* __restrict__ a, long long c, int nv, const T v[4]) {
  if (VEC && nv == 4) {
    typename V4T<T>::t q;
    q.x = v[0]; q.y = v[1]; q.z = v[2]; q.w = v[3];
    *reinterpret_cast<typename V4T<T>::t*>(a + c) = q;
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (e < nv) a[c + e] = v[e];
  }
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

// geometry of one tile and of this thread's quad and halo point
struct QuadGeo {
  int n, i, j, nv, kb, ke;  // quad starts at (i, j); nv valid points; z-range [kb, ke]
  int lx, ly;
  int bxf[5];               // x faces i-1..i+3 (table index without the z code)
  int bym[4], byp[4], bz[4];
  // halo point of this thread (threads 0..127), -1 when none / outside
  int hslot, hi, hj;
  int hb[6];                // the halo point's six face bases (x-,x+,y-,y+ with node z code, z)
};

__device__ __forceinline__ void quad_geo(QuadGeo& G, const ProbDev& P, int tile) {
  const GridDev& g = P.g;
  const int n = g.n;
  G.n = n;
  const int tx = tile % P.ntx, ty = (tile / P.ntx) % P.nty, tz = tile / (P.ntx * P.nty);
  const int t = threadIdx.x;
  G.lx = t & 7;
  G.ly = t >> 3;
  const int i0 = tx * QX + 1, j0 = ty * QY + 1;
  G.i = i0 + 4 * G.lx;
  G.j = j0 + G.ly;
  G.nv = G.j <= n ? max(0, min(4, n - G.i + 1)) : 0;
  G.kb = tz * P.TZ + 1;
  G.ke = min(n, (tz + 1) * P.TZ);
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  const int oY = g.ndir == 3 ? g.nclass : 0, oZ = g.ndir == 3 ? 2 * g.nclass : 0;
  const int jj = min(G.j, n);
  const int cyn = g.code[1][0][jj - 1], cym = g.code[1][1][jj - 1], cyp = g.code[1][1][jj];
#pragma unroll
  for (int e = 0; e < 5; e++) {
    const int f = min(G.i - 1 + e, n);  // face index
    G.bxf[e] = (g.code[0][1][f] * N1 + cyn) * N2;
  }
#pragma unroll
  for (int e = 0; e < 4; e++) {
    const int ii = min(G.i + e, n);
    const int cxn = g.code[0][0][ii - 1];
    G.bym[e] = oY + (cxn * N1 + cym) * N2;
    G.byp[e] = oY + (cxn * N1 + cyp) * N2;
    G.bz[e] = oZ + (cxn * N1 + cyn) * N2;
  }
  // halo: threads 0-31 row j0-1, 32-63 row j0+QY, 64-95 column i0-1, 96-127 column i0+QX
  G.hslot = -1;
  G.hi = G.hj = 0;
  if (t < 128) {
    const int side = t >> 5, o = t & 31;
    int hi, hj, slot;
    if (side == 0) { hi = i0 + o; hj = j0 - 1; slot = o; }
    else if (side == 1) { hi = i0 + o; hj = j0 + QY; slot = (QROWS - 1) * QS + o; }
    else if (side == 2) { hi = i0 - 1; hj = j0 + o; slot = QROWS * QS + 1 + o; }
    else { hi = i0 + QX; hj = j0 + o; slot = QROWS * QS + QROWS + 1 + o; }
    // points outside the grid keep the value 0; the slot is still written
    G.hslot = slot;
    if (hi >= 1 && hi <= n && hj >= 1 && hj <= n) {
      G.hi = hi;
      G.hj = hj;
      const int cxn = g.code[0][0][hi - 1], cxm = g.code[0][1][hi - 1], cxp = g.code[0][1][hi];
      const int hyn = g.code[1][0][hj - 1], hym = g.code[1][1][hj - 1], hyp = g.code[1][1][hj];
      G.hb[0] = (cxm * N1 + hyn) * N2;
      G.hb[1] = (cxp * N1 + hyn) * N2;
      G.hb[2] = oY + (cxn * N1 + hym) * N2;
      G.hb[3] = oY + (cxn * N1 + hyp) * N2;
      G.hb[4] = oZ + (cxn * N1 + hyn) * N2;
      G.hb[5] = 0;
    }
  }
}

// the six coefficients of quad point e at plane k (z codes czn, czm, czp)
template <typename T>
__device__ __forceinline__ void quad_kappa(const QuadGeo& G, const T* kt, int e, int czn, int czm, int czp,
                                           T kk[6]) {
  kk[0] = kt[G.bxf[e] + czn];
  kk[1] = kt[G.bxf[e + 1] + czn];
  kk[2] = kt[G.bym[e] + czn];
  kk[3] = kt[G.byp[e] + czn];
  kk[4] = kt[G.bz[e] + czm];
  kk[5] = kt[G.bz[e] + czp];
}

template <typename T>
__device__ __forceinline__ T diag6T(const T kk[6]) {
  return ((((kk[0] + kk[1]) + kk[2]) + kk[3]) + kk[4]) + kk[5];
}

// policy for the inner products of a sweep
template <typename T> struct DotAcc;
template <> struct DotAcc<double> {  // correctly rounded (FP64 path)
  CrAcc a;
  __device__ __forceinline__ void zero() { a = cr_zero(); }
  __device__ __forceinline__ void add(double x, double y) { cr_add_prod(a, x, y); }
};
template <> struct DotAcc<float> {  // FP64 accumulation of exact float products
  double a;
  __device__ __forceinline__ void zero() { a = 0.0; }
  __device__ __forceinline__ void add(float x, float y) { a = __fma_rn((double)x, (double)y, a); }
};

enum { FOP_AP = 0, FOP_UP2 = 1, FOP_SPMV = 2 };  // SPMV: X = A Pn

// Shared body.  X is x (FP64 CG) or d (FP32 refinement); first_x: X = alpha p.
template <typename T, bool VEC, int OP>
__device__ __forceinline__ void fast_body(const QuadGeo& G, const GridDev& g, const T* kt, T* plane,
                                          const T* __restrict__ R0, T* __restrict__ R, const T* __restrict__ Pold,
                                          T* __restrict__ Pn, T* __restrict__ X, T alpha, T beta, int restart,
                                          int prec, int first_x, DotAcc<T>& a0, DotAcc<T>& a1) {
  const int n = G.n;
  const long long n2 = (long long)n * n;
  const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);  // + (k-1) n^2
  const int nv = G.nv;

  // p_new of the own quad at plane k (AP) or p_new loaded (UP2)
  auto quad_p = [&](int k, T out[4]) {
    if (nv == 0) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = T(0);
      return;
    }
    const long long c = (long long)(k - 1) * n2 + rowoff;
    if (OP != FOP_AP) {
      ld4<T, VEC>(Pn, c, nv, out);
      return;
    }
    T rv[4], po[4];
    ld4<T, VEC>(R0, c, nv, rv);
    if (!restart) ld4<T, VEC>(Pold, c, nv, po);
    const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      T sv = rv[e];
      if (prec) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        sv = rv[e] / diag6T<T>(kk);
      }
      out[e] = (e < nv) ? (restart ? sv : fmaT(beta, po[e], sv)) : T(0);
    }
  };
  // p_new at this thread's halo point of plane k
  auto halo_p = [&](int k) -> T {
    if (G.hi == 0) return T(0);
    const long long c = (long long)(k - 1) * n2 + (long long)(G.hj - 1) * n + (G.hi - 1);
    if (OP != FOP_AP) return Pn[c];
    const T rv = R0[c];
    T sv = rv;
    if (prec) {
      const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
      T kk[6] = {kt[G.hb[0] + czn], kt[G.hb[1] + czn], kt[G.hb[2] + czn],
                 kt[G.hb[3] + czn], kt[G.hb[4] + czm], kt[G.hb[4] + czp]};
      sv = rv / diag6T<T>(kk);
    }
    return restart ? sv : fmaT(beta, Pold[c], sv);
  };

  T pm[4], pc[4], pn[4];
  if (G.kb > 1) quad_p(G.kb - 1, pm);
  else {
#pragma unroll
    for (int e = 0; e < 4; e++) pm[e] = T(0);
  }
  quad_p(G.kb, pc);
  if (OP == FOP_AP && nv > 0) st4<T, VEC>(Pn, (long long)(G.kb - 1) * n2 + rowoff, nv, pc);
  int buf = 0;
  const int mrow = (G.ly + 1) * QS + 4 * G.lx;
  const int hl = QROWS * QS + G.ly + 1, hr = QROWS * QS + QROWS + G.ly + 1;
  for (int k = G.kb; k <= G.ke; k++) {
    if (k < n) {
      quad_p(k + 1, pn);
      if (OP == FOP_AP && k + 1 <= G.ke && nv > 0) st4<T, VEC>(Pn, (long long)k * n2 + rowoff, nv, pn);
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++) pn[e] = T(0);
    }
    T* pl = plane + buf * QPLANE;
#pragma unroll
    for (int e = 0; e < 4; e++) pl[mrow + e] = pc[e];
    if (G.hslot >= 0) pl[G.hslot] = halo_p(k);
    __syncthreads();
    if (nv > 0) {
      const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
      const T left = G.lx > 0 ? pl[mrow - 1] : pl[hl];
      const T right = G.lx < 7 ? pl[mrow + 4] : pl[hr];
      const long long c = (long long)(k - 1) * n2 + rowoff;
      T xo[4], ro[4];
      if (OP == FOP_UP2) {
        if (!first_x) ld4<T, VEC>(X, c, nv, xo);
        ld4<T, VEC>(R, c, nv, ro);
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        const T dg = diag6T<T>(kk);
        const T xm = e > 0 ? pc[e - 1] : left;
        const T xp = e < 3 ? pc[e + 1] : right;
        const T ym = pl[mrow - QS + e], yp = pl[mrow + QS + e];
        T q = dg * pc[e];
        q = fmaT(-kk[0], xm, q);
        q = fmaT(-kk[1], xp, q);
        q = fmaT(-kk[2], ym, q);
        q = fmaT(-kk[3], yp, q);
        q = fmaT(-kk[4], pm[e], q);
        q = fmaT(-kk[5], pn[e], q);
        if (OP == FOP_SPMV) {
          xo[e] = q;
        } else if (e < nv) {
          if (OP == FOP_AP) {
            a0.add(pc[e], q);
          } else {
            xo[e] = first_x ? alpha * pc[e] : fmaT(alpha, pc[e], xo[e]);
            const T rv = fmaT(-alpha, q, ro[e]);
            ro[e] = rv;
            a0.add(rv, rv);
            if (prec) a1.add(rv, rv / dg);
          }
        }
      }
      if (OP == FOP_UP2) {
        st4<T, VEC>(X, c, nv, xo);
        st4<T, VEC>(R, c, nv, ro);
      }
      if (OP == FOP_SPMV) st4<T, VEC>(X, c, nv, xo);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
      pm[e] = pc[e];
      pc[e] = pn[e];
    }
    buf ^= 1;
  }
}

}  // namespace rbws
