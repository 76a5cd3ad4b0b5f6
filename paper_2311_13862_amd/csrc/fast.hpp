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

// Tile shapes: 4 x-points per thread, TPR threads per row, 256 / TPR rows.
// TPR = 8 (32 x 32 columns, halo on all four sides) in general; when one
// tile spans a whole row (32 < n <= 128: TPR 16 or 32, 64 x 16 or 128 x 8
// columns) there is no x-halo and the y-halo rows are contiguous.
constexpr int QX = 32, QY = 32;  // the general shape
// LDS plane: (rows + 2) rows of stride TX + 4, then the left and right halo
// columns; sized for the largest shape (128 x 8: 10 * 132 + 20).
constexpr int QPLANE = 1340;

// Persistent grid over a work list: blocks are dealt round-robin to the 8
// XCDs, so every XCD takes a contiguous share of the list and the tiles of
// one solve (contiguous in the list) share one L2.  gridDim.x is a multiple
// of 8.  `list` == nullptr means all items 0..total-1.
struct WorkRange {
  int w, w1, step;
};
__device__ __forceinline__ WorkRange work_range(int total) {
  const int x = blockIdx.x & 7, nx = gridDim.x >> 3;
  const int chunk = (total + 7) >> 3;
  const int w0 = x * chunk;
  return WorkRange{w0 + (int)(blockIdx.x >> 3), min(total, w0 + chunk), nx};
}

// Append work items item0 .. item0+n-1 to a list (called by the whole
// workgroup; `slot` is workgroup-shared scratch).  The order of solves in a
// list depends on timing, but every item writes its own partial-result slot
// and the per-solve reductions run in tile order, so results do not.
__device__ __forceinline__ void list_push(int* list, int* cnt, int item0, int n, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(cnt, n);
  __syncthreads();
  const int base = *slot;
  for (int t = threadIdx.x; t < n; t += blockDim.x) list[base + t] = item0 + t;
}

template <typename T> struct V4T;
template <> struct V4T<float> { typedef float4 t; };
template <> struct V4T<double> { typedef double4 t; };

// Vectors of a quad at element alignment only (rows of n % 4 != 0 values):
// the 16-byte memory operations need no more than that on this target.
typedef float ua_f4 __attribute__((ext_vector_type(4), aligned(4)));
typedef double ua_d2 __attribute__((ext_vector_type(2), aligned(8)));
template <typename T>
__device__ __forceinline__ void ua_ld4(const T* p, T v[4]) {
  if constexpr (sizeof(T) == 4) {
    const ua_f4 q = *reinterpret_cast<const ua_f4*>(p);
    v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
  } else {
    const ua_d2 q0 = *reinterpret_cast<const ua_d2*>(p), q1 = *reinterpret_cast<const ua_d2*>(p + 2);
    v[0] = q0[0]; v[1] = q0[1]; v[2] = q1[0]; v[3] = q1[1];
  }
}

// The four values of a quad (nv of them inside the grid, the rest 0): one
// vector access when the quad is full.  With VEC (n % 4 == 0) the quad is
// 16-byte aligned and either empty or full.
template <typename T, bool VEC>
__device__ __forceinline__ void ld4(const T* __restrict__ a, long long c, int nv, T v[4]) {
  if (VEC) {  // nv is 0 or 4 when n % 4 == 0
    if (nv == 4) {
      const typename V4T<T>::t q = *reinterpret_cast<const typename V4T<T>::t*>(a + c);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
  } else if (nv == 4) {
    ua_ld4(a + c, v);
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = e < nv ? a[c + e] : T(0);
  }
}

// store of a value that is not read again soon (streamed past the caches).
// FP32 only: a thread's quad is one 16-byte store, so each instruction writes
// whole lines.  An FP64 quad would be two 16-byte stores, each covering half of
// every lane's 32 bytes; streamed, such stores reached memory as 1.06-1.12
// times the vector's bytes, so FP64 results go through ordinary stores.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <typename T, bool VEC>
__device__ __forceinline__ void st4_stream(T* __restrict__ a, long long c, int nv, const T v[4]) {
  static_assert(sizeof(T) == 4, "streamed quad stores are for 4-byte values");
  if constexpr (VEC) {  // nv is 0 or 4 when n % 4 == 0
    if (nv == 4) {
      const nt_f4 q = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(q, reinterpret_cast<nt_f4*>(a + c));
    }
  } else if (nv == 4) {
    const ua_f4 q = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<ua_f4*>(a + c));
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (e < nv) __builtin_nontemporal_store(v[e], a + c + e);
  }
}

// load of a value read once (streamed past the caches)
template <typename T, bool VEC>
__device__ __forceinline__ void ld4_stream(const T* __restrict__ a, long long c, int nv, T v[4]) {
  if (VEC) {
    if (nv == 4) {
      if constexpr (sizeof(T) == 4) {
        const nt_f4 q = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(a + c));
        v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
      } else {
        const nt_d2 q0 = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(a + c));
        const nt_d2 q1 = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(a + c + 2));
        v[0] = q0[0]; v[1] = q0[1]; v[2] = q1[0]; v[3] = q1[1];
      }
    }
  } else if (nv == 4) {
    if constexpr (sizeof(T) == 4) {
      const ua_f4 q = __builtin_nontemporal_load(reinterpret_cast<const ua_f4*>(a + c));
      v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
    } else {
      const ua_d2 q0 = __builtin_nontemporal_load(reinterpret_cast<const ua_d2*>(a + c));
      const ua_d2 q1 = __builtin_nontemporal_load(reinterpret_cast<const ua_d2*>(a + c + 2));
      v[0] = q0[0]; v[1] = q0[1]; v[2] = q1[0]; v[3] = q1[1];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = e < nv ? __builtin_nontemporal_load(a + c + e) : T(0);
  }
}

template <typename T, bool VEC>
__device__ __forceinline__ void st4(T* __restrict__ a, long long c, int nv, const T v[4]) {
  if constexpr (VEC) {  // nv is 0 or 4 when n % 4 == 0
    if (nv == 4) {
      typename V4T<T>::t q;
      q.x = v[0]; q.y = v[1]; q.z = v[2]; q.w = v[3];
      *reinterpret_cast<typename V4T<T>::t*>(a + c) = q;
    }
  } else if (nv == 4) {
    if constexpr (sizeof(T) == 4) {
      const ua_f4 q = {v[0], v[1], v[2], v[3]};
      *reinterpret_cast<ua_f4*>(a + c) = q;
    } else {
      const ua_d2 q0 = {v[0], v[1]}, q1 = {v[2], v[3]};
      *reinterpret_cast<ua_d2*>(a + c) = q0;
      *reinterpret_cast<ua_d2*>(a + c + 2) = q1;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (e < nv) a[c + e] = v[e];
  }
}

// Point e of a quad that holds points (nv > 0): inside the grid.  With VEC
// (n % 4 == 0) a quad is empty or full, so the test folds away there.
template <bool VEC>
__device__ __forceinline__ bool in_quad(int e, int nv) {
  return VEC || e < nv;
}

// A pointer known to address global memory: loads through it are global_load,
// not flat loads (which also count against the LDS wait counter, so that every
// LDS wait would drain them).  For pointers read from memory, whose address
// space the compiler cannot infer.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}
// the same for stores
template <typename T>
using gptr_w = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr_w<T> as_global_w(T* p) {
  return (gptr_w<T>)p;
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
  // LDS plane layout: row stride, this thread's quad, the left/right halo
  // slots of its row, the last lane of a row, whether x-halo columns exist
  int qs, mrow, hl, hr, lxm;
  bool hx;
  // packed z class codes czn | czm << 8 | czp << 16 of the planes kb-1 .. ke+1
  // (index k - kb + 1), staged in LDS by zk_stage
  const int* zk;
};

// The quad's four values in the LDS plane, one 16-byte LDS operation per four
// floats (two per four doubles).  Row stride and quad offset are multiples of
// four elements and the plane starts 16-byte aligned, so the accesses are
// aligned; four scalar accesses at a four-element stride across the lanes
// would meet four-way bank conflicts.
__device__ __forceinline__ void pl_st4(float* p, const float v[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void pl_st4(double* p, const double v[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}
__device__ __forceinline__ void pl_ld4(const float* p, float v[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void pl_ld4(const double* p, double v[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

// A value from the previous lane (lane i reads lane i - 1) or the next one
// (lane i reads lane i + 1): the whole-wave DPP shifts by one lane (GFX9
// wave_shr:1 / wave_shl:1), a VALU move instead of an LDS permute.  The lane
// at the wave's end, which has no source, gets 0.
__device__ __forceinline__ int lane_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int lane_next(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(lane_prev(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(lane_next(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_prev((int)(unsigned)b), hi = lane_prev((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_next((int)(unsigned)b), hi = lane_next((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// x neighbours of the quad whose values c[0..3] are in the plane: the last
// point of the previous quad and the first of the next, taken from the
// neighbouring lanes of the same row (a row is a run of lxm + 1 lanes inside
// one wave), else the x-halo column or the boundary zero.  Every lane of the
// wave must call this (the shifts read the neighbours' registers).
template <typename T>
__device__ __forceinline__ void quad_xnb(const QuadGeo& G, const T* pl, const T c[4], T& left, T& right) {
  const T l = lane_prev(c[3]), r = lane_next(c[0]);
  left = G.lx > 0 ? l : (G.hx ? pl[G.hl] : T(0));
  right = G.lx < G.lxm ? r : (G.hx ? pl[G.hr] : T(0));
}

// Deepest tile (planes per z-march) and the length of its staged z codes.
constexpr int kTzMax = 64;
constexpr int kZkLen = kTzMax + 4;

__device__ __forceinline__ void quad_geo(QuadGeo& G, const ProbDev& P, int tile) {
  const GridDev& g = P.g;
  const int n = g.n;
  G.n = n;
  const int tx = tile % P.ntx, ty = (tile / P.ntx) % P.nty, tz = tile / (P.ntx * P.nty);
  const int t = threadIdx.x;
  const int TX = P.TX, TY = P.TY, tpr = TX >> 2, rows = TY + 2;
  G.lx = t & (tpr - 1);
  G.ly = t / tpr;
  G.lxm = tpr - 1;
  G.qs = TX + 4;
  G.mrow = (G.ly + 1) * G.qs + 4 * G.lx;
  G.hl = rows * G.qs + G.ly + 1;
  G.hr = rows * G.qs + rows + G.ly + 1;
  G.hx = P.ntx > 1 || TX == QX;
  const int i0 = tx * TX + 1, j0 = ty * TY + 1;
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
  // halo.  32 x 32: threads 0-31 row j0-1, 32-63 row j0+TY, 64-95 column i0-1,
  // 96-127 column i0+TX.  Whole-row tiles: threads 0..TX-1 row j0-1, TX..2TX-1
  // row j0+TY (the x-halo lies outside the grid and is never read).
  G.hslot = -1;
  G.hi = G.hj = 0;
  int hi = 0, hj = 0, slot = -1;
  if (TX == QX) {
    if (t < 128) {
      const int side = t >> 5, o = t & 31;
      if (side == 0) { hi = i0 + o; hj = j0 - 1; slot = o; }
      else if (side == 1) { hi = i0 + o; hj = j0 + TY; slot = (rows - 1) * G.qs + o; }
      else if (side == 2) { hi = i0 - 1; hj = j0 + o; slot = rows * G.qs + 1 + o; }
      else { hi = i0 + TX; hj = j0 + o; slot = rows * G.qs + rows + 1 + o; }
    }
  } else if (t < 2 * TX) {
    const int o = t % TX;
    hi = i0 + o;
    if (t < TX) { hj = j0 - 1; slot = o; }
    else { hj = j0 + TY; slot = (rows - 1) * G.qs + o; }
  }
  if (slot >= 0) {
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
// The z-march is software-pipelined: loads for plane k+2 (own quad) and for
// plane k+1 (halo point, x and r) are issued before plane k is consumed.
template <typename T, bool VEC, int OP>
__device__ __forceinline__ void fast_body(const QuadGeo& G, const GridDev& g, const T* kt, T* plane,
                                          const T* __restrict__ R0, T* __restrict__ R, const T* __restrict__ Pold,
                                          T* __restrict__ Pn, T* __restrict__ X, T alpha, T beta, int restart,
                                          int prec, int first_x, DotAcc<T>& a0, DotAcc<T>& a1) {
  const int n = G.n;
  const long long n2 = (long long)n * n;
  const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);  // + (k-1) n^2
  const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);
  const int nv = G.nv;
  const bool hin = G.hi != 0;

  // raw loads of the own quad at plane k: r and p_old (AP) or p_new (UP2/SPMV)
  auto quad_load = [&](int k, T ra[4], T rb[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; e++) ra[e] = rb[e] = T(0);
    if (nv == 0 || k < 1 || k > n) return;
    const long long c = (long long)(k - 1) * n2 + rowoff;
    if (OP != FOP_AP) {
      ld4<T, VEC>(Pn, c, nv, ra);
      return;
    }
    ld4<T, VEC>(R0, c, nv, ra);
    if (!restart) ld4<T, VEC>(Pold, c, nv, rb);
  };
  // p_new of the own quad at plane k from its raw loads
  auto quad_finish = [&](int k, const T ra[4], const T rb[4], T out[4]) __attribute__((always_inline)) {
    if (OP != FOP_AP || nv == 0 || k < 1 || k > n) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = ra[e];
      return;
    }
    const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      T sv = ra[e];
      if (prec) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        sv = ra[e] / diag6T<T>(kk);
      }
      out[e] = in_quad<VEC>(e, nv) ? (restart ? sv : fmaT(beta, rb[e], sv)) : T(0);
    }
  };
  auto halo_load = [&](int k, T& ha, T& hb) __attribute__((always_inline)) {
    ha = hb = T(0);
    if (!hin || k > n) return;
    const long long c = (long long)(k - 1) * n2 + hoff;
    if (OP != FOP_AP) {
      ha = Pn[c];
      return;
    }
    ha = R0[c];
    if (!restart) hb = Pold[c];
  };
  auto halo_finish = [&](int k, T ha, T hb) __attribute__((always_inline)) -> T {
    if (OP != FOP_AP || !hin) return ha;
    T sv = ha;
    if (prec) {
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
      T kk[6] = {kt[G.hb[0] + czn], kt[G.hb[1] + czn], kt[G.hb[2] + czn],
                 kt[G.hb[3] + czn], kt[G.hb[4] + czm], kt[G.hb[4] + czp]};
      sv = ha / diag6T<T>(kk);
    }
    return restart ? sv : fmaT(beta, hb, sv);
  };
  auto xr_load = [&](int k, T xo[4], T ro[4]) __attribute__((always_inline)) {
    if (OP != FOP_UP2 || nv == 0 || k > G.ke) return;
    const long long c = (long long)(k - 1) * n2 + rowoff;
    if (!first_x) ld4<T, VEC>(X, c, nv, xo);
    ld4<T, VEC>(R, c, nv, ro);
  };

  T pm[4], pc[4], pn[4], ra[4], rb[4];
  {
    T qa[4], qb[4];
    quad_load(G.kb - 1, qa, qb);
    quad_finish(G.kb - 1, qa, qb, pm);
    quad_load(G.kb, qa, qb);
    quad_finish(G.kb, qa, qb, pc);
    quad_load(G.kb + 1, qa, qb);
    quad_finish(G.kb + 1, qa, qb, pn);
  }
  if (OP == FOP_AP && nv > 0) {
    st4<T, VEC>(Pn, (long long)(G.kb - 1) * n2 + rowoff, nv, pc);
    if (G.kb + 1 <= G.ke) st4<T, VEC>(Pn, (long long)G.kb * n2 + rowoff, nv, pn);
  }
  T ha, hb, xo[4], ro[4];
  halo_load(G.kb, ha, hb);
#pragma unroll
  for (int e = 0; e < 4; e++) xo[e] = ro[e] = T(0);
  xr_load(G.kb, xo, ro);
  int buf = 0;
  const int mrow = G.mrow;
  for (int k = G.kb; k <= G.ke; k++) {
    // issue the next loads
    quad_load(k + 2, ra, rb);
    T ha2, hb2, xo2[4], ro2[4];
    halo_load(k + 1, ha2, hb2);
#pragma unroll
    for (int e = 0; e < 4; e++) xo2[e] = ro2[e] = T(0);
    xr_load(k + 1, xo2, ro2);
    // consume plane k
    T* pl = plane + buf * QPLANE;
    pl_st4(pl + mrow, pc);
    if (G.hslot >= 0) pl[G.hslot] = halo_finish(k, ha, hb);
    __syncthreads();
    T left, right;
    quad_xnb<T>(G, pl, pc, left, right);
    if (nv > 0) {
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
      T ymv[4], ypv[4];
      pl_ld4(pl + mrow - G.qs, ymv);
      pl_ld4(pl + mrow + G.qs, ypv);
      T qo[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        const T dg = diag6T<T>(kk);
        const T xm = e > 0 ? pc[e - 1] : left;
        const T xp = e < 3 ? pc[e + 1] : right;
        const T ym = ymv[e], yp = ypv[e];
        T q = dg * pc[e];
        q = fmaT(-kk[0], xm, q);
        q = fmaT(-kk[1], xp, q);
        q = fmaT(-kk[2], ym, q);
        q = fmaT(-kk[3], yp, q);
        q = fmaT(-kk[4], pm[e], q);
        q = fmaT(-kk[5], pn[e], q);
        qo[e] = q;
        if (OP != FOP_SPMV && in_quad<VEC>(e, nv)) {
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
      const long long c = (long long)(k - 1) * n2 + rowoff;
      // FP32: x (read again only by the next update) and the product are streamed.
      // FP64: a quad is two 16-byte stores per lane, each instruction covering half
      // of every lane's 32 bytes; streamed, such stores reached memory as 1.12
      // times the vector's bytes (SpMV), as ordinary stores exactly once
      constexpr bool nt = sizeof(T) == 4;
      if (OP == FOP_UP2) {
        if constexpr (nt) st4_stream<T, VEC>(X, c, nv, xo);
        else st4<T, VEC>(X, c, nv, xo);
        st4<T, VEC>(R, c, nv, ro);
      }
      if (OP == FOP_SPMV) {
        if constexpr (nt) st4_stream<T, VEC>(X, c, nv, qo);
        else st4<T, VEC>(X, c, nv, qo);
      }
    }
    // rotate; finish p_new of plane k+2 and store it when it is ours
#pragma unroll
    for (int e = 0; e < 4; e++) {
      pm[e] = pc[e];
      pc[e] = pn[e];
      xo[e] = xo2[e];
      ro[e] = ro2[e];
    }
    quad_finish(k + 2, ra, rb, pn);
    if (OP == FOP_AP && nv > 0 && k + 2 <= G.ke) st4<T, VEC>(Pn, (long long)(k + 1) * n2 + rowoff, nv, pn);
    ha = ha2;
    hb = hb2;
    buf ^= 1;
  }
}

// ---------------------------------------------------------------------------
// FP32 variant of the sweeps.  The face coefficients of the own quad, its
// diagonal and the diagonal's reciprocal are kept in registers and refreshed
// only when the plane's z codes change (the codes are the same for the whole
// block, so the test does not diverge); Jacobi is s = r * (1/d).
// ---------------------------------------------------------------------------
struct KCache32 {
  int key;
  float kx[5], kym[4], kyp[4], kzm[4], kzp[4], dg[4], inv[4];
  float hinv;
};

__device__ __forceinline__ int zkey(const GridDev& g, int k) {
  return g.code[2][0][k - 1] | (g.code[2][1][k - 1] << 8) | (g.code[2][1][k] << 16);
}

// Stages the tile's z codes in LDS (zk[kZkLen], before the barrier that
// publishes the class table).  The z-march then reads them from LDS: a global
// load of a code inside the march would make the wait for it also drain the
// loads issued ahead for later planes.
__device__ __forceinline__ void zk_stage(int* zk, const GridDev& g, QuadGeo& G) {
  for (int t = threadIdx.x; t < G.ke - G.kb + 3; t += blockDim.x) {
    const int k = G.kb - 1 + t;
    zk[t] = (k >= 1 && k <= g.n) ? zkey(g, k) : 0;
  }
  G.zk = zk;
}

__device__ __forceinline__ void kc_fill(KCache32& C, const QuadGeo& G, const float* kt, int key) {
  const int czn = key & 255, czm = (key >> 8) & 255, czp = key >> 16;
#pragma unroll
  for (int e = 0; e < 5; e++) C.kx[e] = kt[G.bxf[e] + czn];
#pragma unroll
  for (int e = 0; e < 4; e++) {
    C.kym[e] = kt[G.bym[e] + czn];
    C.kyp[e] = kt[G.byp[e] + czn];
    C.kzm[e] = kt[G.bz[e] + czm];
    C.kzp[e] = kt[G.bz[e] + czp];
    C.dg[e] = ((((C.kx[e] + C.kx[e + 1]) + C.kym[e]) + C.kyp[e]) + C.kzm[e]) + C.kzp[e];
    C.inv[e] = 1.0f / C.dg[e];
  }
  C.hinv = 1.0f;
  if (G.hi != 0) {
    const float hd = ((((kt[G.hb[0] + czn] + kt[G.hb[1] + czn]) + kt[G.hb[2] + czn]) + kt[G.hb[3] + czn]) +
                      kt[G.hb[4] + czm]) + kt[G.hb[4] + czp];
    C.hinv = 1.0f / hd;
  }
  C.key = key;
}

template <bool VEC, int OP>
__device__ __forceinline__ void fast_body32(const QuadGeo& G, const GridDev& g, const float* kt, float* plane,
                                            const float* __restrict__ R0, float* __restrict__ R,
                                            const float* __restrict__ Pold, float* __restrict__ Pn,
                                            float* __restrict__ X, float alpha, float beta, int restart, int prec,
                                            int first_x, double& a0, double& a1) {
  const int n = G.n;
  const long long n2 = (long long)n * n;
  const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);
  const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);
  const int nv = G.nv;
  const bool hin = G.hi != 0;
  KCache32 C;
  C.key = -1;

  auto quad_load = [&](int k, float ra[4], float rb[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; e++) ra[e] = rb[e] = 0.0f;
    if (nv == 0 || k < 1 || k > n) return;
    const long long c = (long long)(k - 1) * n2 + rowoff;
    if (OP != FOP_AP) {
      ld4<float, VEC>(Pn, c, nv, ra);
      return;
    }
    ld4<float, VEC>(R0, c, nv, ra);
    if (!restart) ld4_stream<float, VEC>(Pold, c, nv, rb);  // the old direction is read once
  };
  // reciprocal diagonal of the own quad at plane k (from the cache when the codes match)
  auto quad_inv = [&](int k, float inv[4]) __attribute__((always_inline)) {
    const int key = G.zk[k - G.kb + 1];
    if (key == C.key) {
#pragma unroll
      for (int e = 0; e < 4; e++) inv[e] = C.inv[e];
      return;
    }
    KCache32 T2;
    kc_fill(T2, G, kt, key);
#pragma unroll
    for (int e = 0; e < 4; e++) inv[e] = T2.inv[e];
  };
  auto quad_finish = [&](int k, const float ra[4], const float rb[4], float out[4]) __attribute__((always_inline)) {
    if (OP != FOP_AP || nv == 0 || k < 1 || k > n) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = ra[e];
      return;
    }
    float inv[4] = {1.0f, 1.0f, 1.0f, 1.0f};
    if (prec) quad_inv(k, inv);
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const float sv = prec ? ra[e] * inv[e] : ra[e];
      out[e] = in_quad<VEC>(e, nv) ? (restart ? sv : fmaf(beta, rb[e], sv)) : 0.0f;
    }
  };
  auto halo_load = [&](int k, float& ha, float& hb) __attribute__((always_inline)) {
    ha = hb = 0.0f;
    if (!hin || k > n) return;
    const long long c = (long long)(k - 1) * n2 + hoff;
    if (OP != FOP_AP) {
      ha = Pn[c];
      return;
    }
    ha = R0[c];
    if (!restart) hb = Pold[c];
  };
  auto xr_load = [&](int k, float xo[4], float ro[4]) __attribute__((always_inline)) {
    if (OP != FOP_UP2 || nv == 0 || k > G.ke) return;
    const long long c = (long long)(k - 1) * n2 + rowoff;
    if (!first_x) ld4_stream<float, VEC>(X, c, nv, xo);  // d is read once
    ld4<float, VEC>(R, c, nv, ro);
  };

  // Loads in flight are never copied between registers (a copy would wait for
  // them): slot S[k & 1] holds the raw quad of plane k+2 and the halo, x and r
  // of plane k, and iteration k fills the other slot with the halo, x and r of
  // plane k+1 and then the quad of plane k+3, which is finished only at the
  // end of iteration k+1.  The loop runs two planes per trip with the slots'
  // roles swapped, so every slot access has a fixed register.
  struct Slot {
    float ra[4], rb[4], ha, hb, xo[4], ro[4];
  };
  Slot S0, S1;
  float pm[4], pc[4], pn[4];
  {
    float qa[4], qb[4];
    quad_load(G.kb - 1, qa, qb);
    quad_finish(G.kb - 1, qa, qb, pm);
    quad_load(G.kb, qa, qb);
    quad_finish(G.kb, qa, qb, pc);
    quad_load(G.kb + 1, qa, qb);
    quad_finish(G.kb + 1, qa, qb, pn);
  }
  if (OP == FOP_AP && nv > 0) {
    st4<float, VEC>(Pn, (long long)(G.kb - 1) * n2 + rowoff, nv, pc);
    if (G.kb + 1 <= G.ke) st4<float, VEC>(Pn, (long long)G.kb * n2 + rowoff, nv, pn);
  }
  halo_load(G.kb, S0.ha, S0.hb);
#pragma unroll
  for (int e = 0; e < 4; e++) S0.xo[e] = S0.ro[e] = 0.0f;
  xr_load(G.kb, S0.xo, S0.ro);
  quad_load(G.kb + 2, S0.ra, S0.rb);
  const int mrow = G.mrow;
  auto iter = [&](int k, Slot& cur, Slot& nxt) __attribute__((always_inline)) {
    halo_load(k + 1, nxt.ha, nxt.hb);
#pragma unroll
    for (int e = 0; e < 4; e++) nxt.xo[e] = nxt.ro[e] = 0.0f;
    xr_load(k + 1, nxt.xo, nxt.ro);
    quad_load(k + 3, nxt.ra, nxt.rb);
    const int key = G.zk[k - G.kb + 1];
    if (key != C.key) kc_fill(C, G, kt, key);
    float* pl = plane + (k & 1) * QPLANE;
    pl_st4(pl + mrow, pc);
    if (G.hslot >= 0) {
      float hv = cur.ha;
      if (OP == FOP_AP && hin) {
        const float sv = prec ? cur.ha * C.hinv : cur.ha;
        hv = restart ? sv : fmaf(beta, cur.hb, sv);
      }
      pl[G.hslot] = hv;
    }
    __syncthreads();
    float left, right;
    quad_xnb<float>(G, pl, pc, left, right);
    if (nv > 0) {
      float ymv[4], ypv[4];
      pl_ld4(pl + mrow - G.qs, ymv);
      pl_ld4(pl + mrow + G.qs, ypv);
      float qo[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const float xm = e > 0 ? pc[e - 1] : left;
        const float xp = e < 3 ? pc[e + 1] : right;
        const float ym = ymv[e], yp = ypv[e];
        float q = C.dg[e] * pc[e];
        q = fmaf(-C.kx[e], xm, q);
        q = fmaf(-C.kx[e + 1], xp, q);
        q = fmaf(-C.kym[e], ym, q);
        q = fmaf(-C.kyp[e], yp, q);
        q = fmaf(-C.kzm[e], pm[e], q);
        q = fmaf(-C.kzp[e], pn[e], q);
        qo[e] = q;
        if (OP != FOP_SPMV && in_quad<VEC>(e, nv)) {
          if (OP == FOP_AP) {
            a0 = __fma_rn((double)pc[e], (double)q, a0);
          } else {
            cur.xo[e] = first_x ? alpha * pc[e] : fmaf(alpha, pc[e], cur.xo[e]);
            const float rv = fmaf(-alpha, q, cur.ro[e]);
            cur.ro[e] = rv;
            a0 = __fma_rn((double)rv, (double)rv, a0);
            if (prec) a1 = __fma_rn((double)rv, (double)(rv * C.inv[e]), a1);
          }
        }
      }
      const long long c = (long long)(k - 1) * n2 + rowoff;
      if (OP == FOP_UP2) {  // d is read again only by the next update or outer pass: streamed
        st4_stream<float, VEC>(X, c, nv, cur.xo);
        st4<float, VEC>(R, c, nv, cur.ro);
      }
      if (OP == FOP_SPMV) st4_stream<float, VEC>(X, c, nv, qo);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
      pm[e] = pc[e];
      pc[e] = pn[e];
    }
    quad_finish(k + 2, cur.ra, cur.rb, pn);
    if (OP == FOP_AP && nv > 0 && k + 2 <= G.ke) st4<float, VEC>(Pn, (long long)(k + 1) * n2 + rowoff, nv, pn);
  };
  int k = G.kb;
  for (; k + 1 <= G.ke; k += 2) {
    iter(k, S0, S1);
    iter(k + 1, S1, S0);
  }
  if (k <= G.ke) iter(k, S0, S1);
}

// ---------------------------------------------------------------------------
// Outer FP64 pass of the refinement on the same tiles: u_new = u + upd d
// (own quad and halo, from u and the FP32 correction d), r = f - A64 u_new in
// the fixed stencil order, b = fl32(r * scale); u_new goes to the other u
// buffer.  Inner products: ||r||^2 (correctly rounded), ||b||^2 and b.P(b).
// ---------------------------------------------------------------------------
template <bool VEC, typename FV>
__device__ __forceinline__ void outer_body(const QuadGeo& G, const GridDev& g, const double* k64, const float* k32,
                                           double* plane, const double* __restrict__ Us, double* __restrict__ Ud,
                                           const float* __restrict__ D, float* __restrict__ R, double upd,
                                           double scale, int prec, int first, FV fv, CrAcc& arr, CrAcc& aff,
                                           double& bb, double& bs) {
  const int n = G.n;
  const long long n2 = (long long)n * n;
  const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);
  const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);
  const int nv = G.nv;
  const bool hin = G.hi != 0;
  const bool up = upd != 0.0;
  auto quad_u = [&](int k, double out[4]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; e++) out[e] = 0.0;
    if (nv == 0 || k < 1 || k > n) return;
    const long long c = (long long)(k - 1) * n2 + rowoff;
    ld4<double, VEC>(Us, c, nv, out);
    if (up) {
      float dv[4] = {0.f, 0.f, 0.f, 0.f};
      ld4<float, VEC>(D, c, nv, dv);
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = in_quad<VEC>(e, nv) ? __fma_rn(upd, (double)dv[e], out[e]) : 0.0;
    }
  };
  auto halo_u = [&](int k) __attribute__((always_inline)) -> double {
    if (!hin || k > n) return 0.0;
    const long long c = (long long)(k - 1) * n2 + hoff;
    return up ? __fma_rn(upd, (double)D[c], Us[c]) : Us[c];
  };
  double um[4], uc[4], un[4];
  quad_u(G.kb - 1, um);
  quad_u(G.kb, uc);
  double hv = halo_u(G.kb);
  int buf = 0;
  const int mrow = G.mrow;
  for (int k = G.kb; k <= G.ke; k++) {
    quad_u(k + 1, un);
    const double hv2 = halo_u(k + 1);
    double* pl = plane + buf * QPLANE;
    pl_st4(pl + mrow, uc);
    if (G.hslot >= 0) pl[G.hslot] = hv;
    __syncthreads();
    double left, right;
    quad_xnb<double>(G, pl, uc, left, right);
    if (nv > 0) {
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
      double ymv[4], ypv[4];
      pl_ld4(pl + mrow - G.qs, ymv);
      pl_ld4(pl + mrow + G.qs, ypv);
      float ro[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        double kk[6];
        quad_kappa<double>(G, k64, e, czn, czm, czp, kk);
        const double xm = e > 0 ? uc[e - 1] : left;
        const double xp = e < 3 ? uc[e + 1] : right;
        double q = diag6T<double>(kk) * uc[e];
        q = __fma_rn(-kk[0], xm, q);
        q = __fma_rn(-kk[1], xp, q);
        q = __fma_rn(-kk[2], ymv[e], q);
        q = __fma_rn(-kk[3], ypv[e], q);
        q = __fma_rn(-kk[4], um[e], q);
        q = __fma_rn(-kk[5], un[e], q);
        ro[e] = 0.0f;
        if (in_quad<VEC>(e, nv)) {
          const double f = fv(G.i + e, G.j, k);
          const double rv = f - q;
          const float r32 = (float)(rv * scale);
          ro[e] = r32;
          cr_add_prod(arr, rv, rv);
          if (first) cr_add_prod(aff, f, f);
          bb = __fma_rn((double)r32, (double)r32, bb);
          if (prec) {
            float k3[6];
            quad_kappa<float>(G, k32, e, czn, czm, czp, k3);
            bs = __fma_rn((double)r32, (double)(r32 / diag6T<float>(k3)), bs);
          }
        }
      }
      const long long c = (long long)(k - 1) * n2 + rowoff;
      st4<float, VEC>(R, c, nv, ro);
      // u' is read again only at the next outer pass, but a streamed FP64 quad (two
      // 16-byte stores per lane, each covering half of every lane's 32 bytes)
      // reached memory as more than u's bytes: ordinary stores (0.90 against 0.95 ms)
      if (up) st4<double, VEC>(Ud, c, nv, uc);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
      um[e] = uc[e];
      uc[e] = un[e];
    }
    hv = hv2;
    buf ^= 1;
  }
}

}  // namespace rbws
