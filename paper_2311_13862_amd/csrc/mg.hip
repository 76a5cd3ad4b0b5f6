// mg.hip -- multigrid V-cycle preconditioner (the paper's Alg. 2) for the
// batched PCG of Alg. 1 (MGCG), in FP64 (reproducible) or FP32 (refinement).
//
// Hierarchy: n_0 = n, n_{l+1} = (n_l - 1) / 2 while n_l > 3.  Every level is
// the same 7-point face rule on its own grid (the paper forms P^T A P; the
// rediscretised operator keeps the matrix-free class-table form on every
// level).  Vertex grids with n+1 intervals are not nested when n+1 is odd, so
// P is trilinear interpolation between them: fine node i (at i/(nf+1)) lies in
// coarse interval I = floor(i (nc+1) / (nf+1)) with weight
// w = (i (nc+1) - I (nf+1)) / (nf+1) on node I+1 and 1 - w on node I; coarse
// boundary nodes carry 0.  R = ((nc+1)/(nf+1)) P^T keeps the coarse right-hand
// side consistent with the unscaled coarse operator.  The coarsest level (at
// most 27 unknowns) is solved by a per-solve dense Cholesky factorisation.
// Smoother: damped Jacobi, nu sweeps before and after the coarse correction.
//
// Kernels are one thread per grid point (per coarse point for the
// restriction, per solve for the coarsest solve), with a fixed evaluation
// order for every value:
//   Jacobi        q = A e (stencil order), t = b - q, t = t / d, e' = fma(omega, t, e)
//   restriction   ax = fma(px, r, ax) over i, ay = fma(py, ax, ay) over j,
//                 az = fma(pz, ay, az) over k (ascending, from 0), then az * scale
//   prolongation  az = fma(wz, e_c, az) over z corners, ay = fma(wy, az, ay) over
//                 y corners, v = fma(wx, ay, v) over x corners (interior ones,
//                 corner 0 then 1, from 0), then e + v
//   coarsest      Cholesky and triangular solves with sequential fma accumulation
// so that the FP64 V-cycle, and with it the whole MGCG trajectory, is
// independent of the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fast.hpp"
#include "mg.hpp"

namespace rbws {

Problem* problem_create(const rbws_problem_desc* d, int device);

int mg_levels_of(int n, int* out) {
  int k = 0;
  out[k++] = n;
  while (out[k - 1] > 3 && k < 16) {
    out[k] = (out[k - 1] - 1) / 2;
    k++;
  }
  return k;
}

// ---------------------------------------------------------------------------
// device views
// ---------------------------------------------------------------------------
struct MgLv {
  const ProbDev* pd;       // the level's grid
  const SolveDev* sd;      // per group solve: offset of its coefficient table
  const void* kap;         // coefficient tables (double or float)
  const long long* voff;   // vector offset per group solve, or null: t * ndof
  const int* sid;          // batch solve of each group solve
  long long ndof;
  int n, nsol;
};

template <typename T>
__device__ __forceinline__ void kappa6(const GridDev& g, const T* kap, int i, int j, int k, T kk[6]) {
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  const T* kX = kap;
  const T* kY = kap + (g.ndir == 3 ? g.nclass : 0);
  const T* kZ = kap + (g.ndir == 3 ? 2 * g.nclass : 0);
  const int cxn = g.code[0][0][i - 1], cxm = g.code[0][1][i - 1], cxp = g.code[0][1][i];
  const int cyn = g.code[1][0][j - 1], cym = g.code[1][1][j - 1], cyp = g.code[1][1][j];
  const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
  kk[0] = kX[(cxm * N1 + cyn) * N2 + czn];
  kk[1] = kX[(cxp * N1 + cyn) * N2 + czn];
  kk[2] = kY[(cxn * N1 + cym) * N2 + czn];
  kk[3] = kY[(cxn * N1 + cyp) * N2 + czn];
  kk[4] = kZ[(cxn * N1 + cyn) * N2 + czm];
  kk[5] = kZ[(cxn * N1 + cyn) * N2 + czp];
}

template <typename T>
__device__ __forceinline__ T stencilT(const T kk[6], T dg, const T* v, long long c, int n, int i, int j, int k) {
  const long long n2 = (long long)n * n;
  T acc = dg * v[c];
  if (i > 1) acc = fmaT(-kk[0], v[c - 1], acc);
  if (i < n) acc = fmaT(-kk[1], v[c + 1], acc);
  if (j > 1) acc = fmaT(-kk[2], v[c - n], acc);
  if (j < n) acc = fmaT(-kk[3], v[c + n], acc);
  if (k > 1) acc = fmaT(-kk[4], v[c - n2], acc);
  if (k < n) acc = fmaT(-kk[5], v[c + n2], acc);
  return acc;
}

template <typename T>
__device__ __forceinline__ T diagT(const T kk[6]) {
  return ((((kk[0] + kk[1]) + kk[2]) + kk[3]) + kk[4]) + kk[5];
}

// ---------------------------------------------------------------------------
// kernels: a grid of workgroups walks the (listed solve, chunk of 256 points)
// items; XCD x (blocks b with b % 8 == x) takes a contiguous eighth of them, so
// the chunks of one solve, which read each other's halo planes, share an L2
// ---------------------------------------------------------------------------
struct MgList {
  const int* list;  // group-local solve indices
  const int* cnt;   // their number
};

// (all index arithmetic below is 32-bit: a level has at most 2^30 points and a
// list at most 2^31 items; 64-bit division would dominate these kernels)
struct ItemRange {
  int w, w1, step;
};
__device__ __forceinline__ ItemRange item_range(int total) {
  const int x = blockIdx.x & 7;
  const int nx = gridDim.x >> 3;
  const int per = (total + 7) >> 3;
  const int w0 = x * per;
  return ItemRange{w0 + (int)(blockIdx.x >> 3), min(total, w0 + per), nx};
}
// e_out = e_in + omega (b - A e_in) / d  (e_in null: zero); RESID: t = b - A e_in
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_mg_point(MgLv L, MgList ml, const T* __restrict__ b,
                                                  const T* __restrict__ ein, T* __restrict__ out, T omega) {
  const int chunks = (int)((L.ndof + 255) >> 8), nd = (int)L.ndof;
  const ItemRange R = item_range(*ml.cnt * chunks);
  const int n = L.n;
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / chunks];
    const int c = (w % chunks) * 256 + (int)threadIdx.x;
    if (c >= nd) continue;
    const int ij = c % (n * n);
    const int i = ij % n + 1, j = ij / n + 1, k = c / (n * n) + 1;
    const long long off = L.voff ? L.voff[t] : (long long)t * L.ndof;
    T kk[6];
    kappa6<T>(L.pd->g, (const T*)L.kap + L.sd[t].kap_off, i, j, k, kk);
    const T dg = diagT(kk);
    const T q = ein ? stencilT<T>(kk, dg, ein + off, c, n, i, j, k) : T(0);
    T r = b[off + c] - q;
    if (RESID) {
      out[off + c] = r;
    } else {
      r = r / dg;
      out[off + c] = fmaT(omega, r, ein ? ein[off + c] : T(0));
    }
  }
}

// Transfers between levels, weights from the tables ci (coarse node left of a
// fine point), cw (its offset) and lohi (fine span of a coarse node).
//
// Restriction b_c = scale P^T r_f, separable as
//   ax[k][j][I] = sum_i px r[k][j][i],  ay = sum_j py ax,  az = sum_k pz ay,
// each an fma chain from 0 over ascending fine index, then b_c = az * scale.
constexpr int kSpan = 6;  // fine points per coarse node and axis: 2 (nf+1)/(nc+1) + 1 <= 6

template <typename T>
__device__ __forceinline__ int fine_weights(int I, const int* __restrict__ ci, const T* __restrict__ cw,
                                            const int2* __restrict__ lohi, T wts[kSpan]) {
  const int2 r = lohi[I];
#pragma unroll
  for (int u = 0; u < kSpan; u++) {
    const int i = r.x + u;
    wts[u] = i <= r.y ? (ci[i - 1] == I ? T(1) - cw[i - 1] : cw[i - 1]) : T(0);
  }
  return r.x;
}

// One pass, a z-march: a block owns a quad of coarse rows J (a wave each), a
// chunk of 64 coarse columns I (a lane each) and a segment of kRsSeg coarse
// planes, and walks the fine planes k that feed them.  Per plane the fine
// block (rows in the quad's span) x (columns in the chunk's span) is staged in
// LDS (loaded one plane ahead into registers), the x-sums ax[j][I] are formed
// there, and each thread forms ay(k) for its (J, I) and adds it to the coarse
// planes K = ci(k) (weight 1 - cw) and ci(k) + 1 (weight cw), in ascending k:
// the order of the chains over k.  With (nc+1)/(nf+1) <= 1/2, ci grows by at
// most one per fine plane, so two accumulators (K = Kc, Kc + 1) suffice and Kc
// is complete once ci has moved past it.
constexpr int kRsSeg = 16;
constexpr int kRsRows = 16;   // fine rows of a J quad's span (checked at set-up)
constexpr int kRsCols = 144;  // fine columns of an I chunk's span (checked at set-up)
constexpr int kRsQ = (kRsCols + 63) / 64;
constexpr int kRsPer = (kRsRows / 4) * kRsQ;  // staged values per thread

template <typename T>
__global__ __launch_bounds__(256) void k_mg_restrict(MgLv F, MgLv C, MgList ml, const int* __restrict__ ci,
                                                     const T* __restrict__ cw, const int2* __restrict__ lohi,
                                                     const T* __restrict__ rf, T* __restrict__ bc, T scale) {
  __shared__ T tile[2][kRsRows][kRsCols];
  __shared__ T axs[2][kRsRows][64];
  const int nc = C.n, nf = F.n;
  const int ich = (nc + 63) >> 6, jq = (nc + 3) >> 2, nseg = (nc + kRsSeg - 1) / kRsSeg;
  const int cols = jq * ich, per = nseg * cols;  // (segment, J quad, I chunk) items per solve
  const ItemRange R = item_range(*ml.cnt * per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nc2 = (long long)nc * nc, nf2 = (long long)nf * nf;
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / per];
    const int rem = w % per, sg = rem / cols, rc = rem % cols;
    const int Jq0 = (rc / ich) * 4 + 1, Iq0 = (rc % ich) * 64 + 1;
    const int J = Jq0 + wv, I = Iq0 + lane;
    const bool act = J <= nc && I <= nc;
    const int Jl = min(Jq0 + 3, nc), Il = min(Iq0 + 63, nc);
    const int jr0 = lohi[Jq0].x, nr = lohi[Jl].y - jr0 + 1;  // staged fine rows
    const int ic0 = lohi[Iq0].x, ncl = lohi[Il].y - ic0 + 1;  // staged fine columns
    const int Ks = sg * kRsSeg + 1, Ke = min(nc, Ks + kRsSeg - 1);
    const int k0 = lohi[Ks].x, k1 = lohi[Ke].y;
    // per-thread weights: x for column I, y for row J
    T wx[kSpan], wy[kSpan];
    const int Ic = min(I, nc), Jc = min(J, nc);
    const int xo = fine_weights(Ic, ci, cw, lohi, wx) - ic0, xn = lohi[Ic].y - lohi[Ic].x + 1;
    const int yo = fine_weights(Jc, ci, cw, lohi, wy) - jr0, yn = lohi[Jc].y - lohi[Jc].x + 1;
    const T* src = rf + (F.voff ? F.voff[t] : (long long)t * F.ndof) + (long long)(jr0 - 1) * nf + (ic0 - 1);
    T* out = bc + (C.voff ? C.voff[t] : (long long)t * C.ndof) + (long long)(Jc - 1) * nc + (Ic - 1);
    T st[kRsPer];
    auto load = [&](int k) __attribute__((always_inline)) {
      const T* p = src + (long long)(k - 1) * nf2;
#pragma unroll
      for (int m = 0; m < kRsRows / 4; m++)
#pragma unroll
        for (int q = 0; q < kRsQ; q++) {
          const int r = wv + 4 * m, c = lane + 64 * q;
          st[m * kRsQ + q] = (r < nr && c < ncl) ? p[(long long)r * nf + c] : T(0);
        }
    };
    int Kc = ci[k0 - 1];
    T accA = T(0), accB = T(0);
    load(k0);
    int buf = 0;
    for (int k = k0; k <= k1; k++) {
#pragma unroll
      for (int m = 0; m < kRsRows / 4; m++)
#pragma unroll
        for (int q = 0; q < kRsQ; q++)
          if (lane + 64 * q < kRsCols) tile[buf][wv + 4 * m][lane + 64 * q] = st[m * kRsQ + q];
      if (k < k1) load(k + 1);
      __syncthreads();
      // x-sums of the staged rows at this lane's column I
#pragma unroll
      for (int m = 0; m < kRsRows / 4; m++) {
        const int r = wv + 4 * m;
        T ax = T(0);
#pragma unroll
        for (int u = 0; u < kSpan; u++)
          if (u < xn) ax = fmaT(wx[u], tile[buf][r][xo + u], ax);
        axs[buf][r][lane] = ax;
      }
      __syncthreads();
      const int K0 = ci[k - 1];
      const T wz = cw[k - 1];
      if (K0 != Kc) {
        if (act && Kc >= Ks) out[(Kc - 1) * nc2] = accA * scale;
        accA = accB;
        accB = T(0);
        Kc = K0;
      }
      T ay = T(0);
#pragma unroll
      for (int u = 0; u < kSpan; u++)
        if (u < yn) ay = fmaT(wy[u], axs[buf][yo + u][lane], ay);
      if (K0 >= 1) accA = fmaT(T(1) - wz, ay, accA);
      if (K0 + 1 <= nc) accB = fmaT(wz, ay, accB);
      buf ^= 1;
    }
    if (act && Kc >= Ks && Kc <= Ke) out[(Kc - 1) * nc2] = accA * scale;
    if (act && Kc + 1 >= Ks && Kc + 1 <= Ke) out[Kc * nc2] = accB * scale;
    __syncthreads();  // LDS of this item is free
  }
}

// The y/z part alone, when the fine level's pre-smoothing has already formed
// the x-sums ax[k][j][I] (fine rows of n_c values, group layout): per fine
// plane the rows of the quad's y-span go to LDS (loaded one plane ahead), then
// the same y and z chains as above.
// The y/z part of the restriction from x-sums ax[k][j][I] (formed by the FP32
// pre-smoothing): a block owns kRyJ = 8 coarse rows J (two per wave, J and
// J + 4), a chunk of 64 coarse columns I (a lane each) and a segment of kRsSeg
// coarse planes.  Per fine plane it stages the rows of the octet's span in LDS
// (loaded one plane ahead into registers); each thread then forms ay(k) for its
// two (J, I) and adds them to the coarse planes K = ci(k) and ci(k) + 1 in
// ascending k, as the one-pass kernel does.  Eight rows per block read about
// 1.2 times the x-sums' rows where four read 1.4 times.
constexpr int kRyJ = 8;      // coarse rows per block
constexpr int kRyRows = 24;  // fine rows of their span (checked at set-up)

template <typename T>
__global__ __launch_bounds__(256) void k_mg_restrict_yz(MgLv F, MgLv C, MgList ml, const int* __restrict__ ci,
                                                        const T* __restrict__ cw, const int2* __restrict__ lohi,
                                                        const T* __restrict__ tx, T* __restrict__ bc, T scale) {
  __shared__ T axs[2][kRyRows][64];
  const int nc = C.n, nf = F.n;
  const int ich = (nc + 63) >> 6, jq = (nc + kRyJ - 1) / kRyJ, nseg = (nc + kRsSeg - 1) / kRsSeg;
  const int cols = jq * ich, per = nseg * cols;  // (segment, J octet, I chunk) items per solve
  const ItemRange R = item_range(*ml.cnt * per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nc2 = (long long)nc * nc, fplane = (long long)nf * nc;
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / per];
    const int rem = w % per, sg = rem / cols, rc = rem % cols;
    const int Jq0 = (rc / ich) * kRyJ + 1, Iq0 = (rc % ich) * 64 + 1;
    const int I = Iq0 + lane;
    const int Jl = min(Jq0 + kRyJ - 1, nc);
    const int jr0 = lohi[Jq0].x, nr = lohi[Jl].y - jr0 + 1;  // staged fine rows
    const int Ks = sg * kRsSeg + 1, Ke = min(nc, Ks + kRsSeg - 1);
    const int k0 = lohi[Ks].x, k1 = lohi[Ke].y;
    const int Ic = min(I, nc);
    const long long vo = C.voff ? C.voff[t] : (long long)t * C.ndof;
    T wy[2][kSpan];
    int yo[2], yn[2];
    bool act[2];
    T* out[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int J = Jq0 + wv + 4 * h;
      const int Jc = min(J, nc);
      act[h] = J <= nc && I <= nc;
      yo[h] = fine_weights(Jc, ci, cw, lohi, wy[h]) - jr0;
      yn[h] = lohi[Jc].y - lohi[Jc].x + 1;
      out[h] = bc + vo + (long long)(Jc - 1) * nc + (Ic - 1);
    }
    const T* src = tx + (long long)t * nf * fplane + (long long)(jr0 - 1) * nc + (Ic - 1);
    T st[kRyRows / 4];
    auto load = [&](int k) __attribute__((always_inline)) {
      const T* p = src + (long long)(k - 1) * fplane;
#pragma unroll
      for (int m = 0; m < kRyRows / 4; m++) {
        const int r = wv + 4 * m;
        st[m] = (r < nr && I <= nc) ? p[(long long)r * nc] : T(0);
      }
    };
    int Kc = ci[k0 - 1];
    T accA[2] = {T(0), T(0)}, accB[2] = {T(0), T(0)};
    load(k0);
    int buf = 0;
    for (int k = k0; k <= k1; k++) {
#pragma unroll
      for (int m = 0; m < kRyRows / 4; m++) axs[buf][wv + 4 * m][lane] = st[m];
      if (k < k1) load(k + 1);
      __syncthreads();
      const int K0 = ci[k - 1];
      const T wz = cw[k - 1];
      if (K0 != Kc) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
          if (act[h] && Kc >= Ks) out[h][(Kc - 1) * nc2] = accA[h] * scale;
          accA[h] = accB[h];
          accB[h] = T(0);
        }
        Kc = K0;
      }
#pragma unroll
      for (int h = 0; h < 2; h++) {
        T ay = T(0);
#pragma unroll
        for (int u = 0; u < kSpan; u++)
          if (u < yn[h]) ay = fmaT(wy[h][u], axs[buf][yo[h] + u][lane], ay);
        if (K0 >= 1) accA[h] = fmaT(T(1) - wz, ay, accA[h]);
        if (K0 + 1 <= nc) accB[h] = fmaT(wz, ay, accB[h]);
      }
      buf ^= 1;
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
      if (act[h] && Kc >= Ks && Kc <= Ke) out[h][(Kc - 1) * nc2] = accA[h] * scale;
      if (act[h] && Kc + 1 >= Ks && Kc + 1 <= Ke) out[h][Kc * nc2] = accB[h] * scale;
    }
    __syncthreads();  // LDS of this item is free
  }
}

// Prolongation, separable: first the coarse values are interpolated in z and y
// onto the fine (k, j) rows at every coarse column I,
//   ezy[k][j][I] = sum_cy wy (sum_cz wz e_c[K][J][I])    (fma chains from 0),
// then each fine point takes v = sum_cx wx ezy[k][j][I0 + cx].  Out-of-grid
// coarse nodes (value 0) are skipped.  The z/y pass is a z-march: a thread owns
// a fine (j, I) column and a segment of kPzSeg fine planes, and keeps the four
// coarse values at (K0, K0 + 1) x (J0, J0 + 1) in registers; when K0 = ci(k)
// advances, the old upper plane becomes the lower one and one plane is loaded.
constexpr int kPzSeg = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_mg_pyz(MgLv F, MgLv C, MgList ml, const int* __restrict__ ci,
                                                const T* __restrict__ cw, const T* __restrict__ ec,
                                                T* __restrict__ ezy) {
  const int nc = C.n, nf = F.n;
  const int ich = (nc + 63) >> 6, jq = (nf + 3) >> 2, nseg = (nf + kPzSeg - 1) / kPzSeg;
  const int cols = jq * ich, per = nseg * cols;  // (segment, j quad, I chunk) items per solve
  const ItemRange R = item_range(*ml.cnt * per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long nc2 = (long long)nc * nc, fplane = (long long)nf * nc;
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / per];
    const int rem = w % per, sg = rem / cols, rc = rem % cols;
    const int j = (rc / ich) * 4 + wv + 1, I = (rc % ich) * 64 + lane + 1;
    if (j > nf || I > nc) continue;
    const int kA = sg * kPzSeg + 1, kB = min(nf, kA + kPzSeg - 1);
    const int J0 = ci[j - 1];
    const T wy1 = cw[j - 1];
    const bool y0 = J0 >= 1, y1 = J0 + 1 <= nc;
    const T* e = ec + (C.voff ? C.voff[t] : (long long)t * C.ndof) + (I - 1);
    T* o = ezy + (long long)t * nf * fplane + (long long)(j - 1) * nc + (I - 1);
    auto plane = [&](int K, T& v0, T& v1) __attribute__((always_inline)) {
      v0 = v1 = T(0);
      if (K < 1 || K > nc) return;
      const T* eK = e + (long long)(K - 1) * nc2;
      if (y0) v0 = eK[(long long)(J0 - 1) * nc];
      if (y1) v1 = eK[(long long)J0 * nc];
    };
    int Kc = ci[kA - 1];
    T a0, a1, b0, b1;  // coarse plane Kc at rows J0, J0 + 1; plane Kc + 1
    plane(Kc, a0, a1);
    plane(Kc + 1, b0, b1);
    for (int k = kA; k <= kB; k++) {
      const int K0 = ci[k - 1];
      if (K0 != Kc) {
        a0 = b0;
        a1 = b1;
        Kc = K0;
        plane(Kc + 1, b0, b1);
      }
      const T wz1 = cw[k - 1];
      T ay = T(0);
      if (y0) {
        T az = T(0);
        if (K0 >= 1) az = fmaT(T(1) - wz1, a0, az);
        if (K0 + 1 <= nc) az = fmaT(wz1, b0, az);
        ay = fmaT(T(1) - wy1, az, ay);
      }
      if (y1) {
        T az = T(0);
        if (K0 >= 1) az = fmaT(T(1) - wz1, a1, az);
        if (K0 + 1 <= nc) az = fmaT(wz1, b1, az);
        ay = fmaT(wy1, az, ay);
      }
      o[(long long)(k - 1) * fplane] = ay;
    }
  }
}

// v = sum over the x corners of wx ezy (row pointer at coarse column 1)
template <typename T>
__device__ __forceinline__ T prolong_x(const T* __restrict__ row, int nc, int I0, T wx1) {
  T v = T(0);
  if (I0 >= 1) v = fmaT(T(1) - wx1, row[I0 - 1], v);
  if (I0 + 1 <= nc) v = fmaT(wx1, row[I0], v);
  return v;
}

// ---------------------------------------------------------------------------
// the same point operations on quads of 4 x-consecutive points (n % 4 == 0,
// 16-byte aligned vectors): one vector load per neighbour plane or row
// instead of four scalar ones.  Out-of-grid neighbours enter as +0, which
// leaves the fma chain bit-identical to skipping them.
// ---------------------------------------------------------------------------
template <typename T>
struct V4 {
  T v[4];
};
template <typename T>
__device__ __forceinline__ V4<T> ld4q(const T* p) {
  V4<T> r;
  if (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    r.v[0] = f.x;
    r.v[1] = f.y;
    r.v[2] = f.z;
    r.v[3] = f.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = a.x;
    r.v[1] = a.y;
    r.v[2] = b.x;
    r.v[3] = b.y;
  }
  return r;
}
template <typename T>
__device__ __forceinline__ void st4q(T* p, const T v[4]) {
  if (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  }
}
template <typename T>
__device__ __forceinline__ V4<T> zero4() {
  V4<T> r;
  r.v[0] = r.v[1] = r.v[2] = r.v[3] = T(0);
  return r;
}

template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_mg_quad(MgLv L, MgList ml, const T* __restrict__ b,
                                                 const T* __restrict__ ein, T* __restrict__ out, T omega) {
  const int n = L.n, nd = (int)L.ndof, nq = nd >> 2;
  const int chunks = (nq + 255) >> 8;
  const ItemRange R = item_range(*ml.cnt * chunks);
  const GridDev& g = L.pd->g;
  const int N1 = g.ncode[1], N2 = g.ncode[2];
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / chunks];
    const int q = (w % chunks) * 256 + (int)threadIdx.x;
    if (q >= nq) continue;
    const int c = q * 4;
    const int ij = c % (n * n);
    const int i0 = ij % n + 1, j = ij / n + 1, k = c / (n * n) + 1;
    const long long off = L.voff ? L.voff[t] : (long long)t * L.ndof;
    const T* kX = (const T*)L.kap + L.sd[t].kap_off;
    const T* kY = kX + (g.ndir == 3 ? g.nclass : 0);
    const T* kZ = kX + (g.ndir == 3 ? 2 * g.nclass : 0);
    const int cyn = g.code[1][0][j - 1], cym = g.code[1][1][j - 1], cyp = g.code[1][1][j];
    const int czn = g.code[2][0][k - 1], czm = g.code[2][1][k - 1], czp = g.code[2][1][k];
    const V4<T> B = ld4q(b + off + c);
    V4<T> E = zero4<T>(), YM = zero4<T>(), YP = zero4<T>(), ZM = zero4<T>(), ZP = zero4<T>();
    T xm = T(0), xp = T(0);
    if (ein) {
      const T* e = ein + off;
      E = ld4q(e + c);
      if (i0 > 1) xm = e[c - 1];
      if (i0 + 3 < n) xp = e[c + 4];
      if (j > 1) YM = ld4q(e + c - n);
      if (j < n) YP = ld4q(e + c + n);
      if (k > 1) ZM = ld4q(e + c - n * n);
      if (k < n) ZP = ld4q(e + c + n * n);
    }
    T o[4];
#pragma unroll
    for (int el = 0; el < 4; el++) {
      const int i = i0 + el;
      const int cxn = g.code[0][0][i - 1], cxm = g.code[0][1][i - 1], cxp = g.code[0][1][i];
      T kk[6];
      kk[0] = kX[(cxm * N1 + cyn) * N2 + czn];
      kk[1] = kX[(cxp * N1 + cyn) * N2 + czn];
      kk[2] = kY[(cxn * N1 + cym) * N2 + czn];
      kk[3] = kY[(cxn * N1 + cyp) * N2 + czn];
      kk[4] = kZ[(cxn * N1 + cyn) * N2 + czm];
      kk[5] = kZ[(cxn * N1 + cyn) * N2 + czp];
      const T dg = diagT(kk);
      T qv = T(0);
      if (ein) {
        qv = dg * E.v[el];
        qv = fmaT(-kk[0], el > 0 ? E.v[el - 1] : xm, qv);
        qv = fmaT(-kk[1], el < 3 ? E.v[el + 1] : xp, qv);
        qv = fmaT(-kk[2], YM.v[el], qv);
        qv = fmaT(-kk[3], YP.v[el], qv);
        qv = fmaT(-kk[4], ZM.v[el], qv);
        qv = fmaT(-kk[5], ZP.v[el], qv);
      }
      T r = B.v[el] - qv;
      if (RESID) {
        o[el] = r;
      } else {
        r = r / dg;
        o[el] = fmaT(omega, r, ein ? E.v[el] : T(0));
      }
    }
    st4q(out + off + c, o);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong_quad(MgLv F, MgLv C, MgList ml, const int* __restrict__ ci,
                                                         const T* __restrict__ cw, const T* __restrict__ ezy,
                                                         T* __restrict__ ef) {
  const int nf = F.n, nc = C.n, nd = (int)F.ndof, nq = nd >> 2;
  const int chunks = (nq + 255) >> 8;
  const ItemRange R = item_range(*ml.cnt * chunks);
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / chunks];
    const int q = (w % chunks) * 256 + (int)threadIdx.x;
    if (q >= nq) continue;
    const int c = q * 4;
    const int i0 = c % nf + 1, row = c / nf;
    const T* zr = ezy + (long long)t * nf * nf * nc + (long long)row * nc;
    T* o = ef + (F.voff ? F.voff[t] : (long long)t * F.ndof) + c;
    V4<T> X = ld4q(o);
#pragma unroll
    for (int el = 0; el < 4; el++) X.v[el] = X.v[el] + prolong_x(zr, nc, ci[i0 + el - 1], cw[i0 + el - 1]);
    st4q(o, X.v);
  }
}

// e_f += P e_c, one thread per fine point (from the z/y-interpolated ezy)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong(MgLv F, MgLv C, MgList ml, const int* __restrict__ ci,
                                                    const T* __restrict__ cw, const T* __restrict__ ezy,
                                                    T* __restrict__ ef) {
  const int nf = F.n, nc = C.n, nd = (int)F.ndof;
  const int chunks = (nd + 255) >> 8;
  const ItemRange R = item_range(*ml.cnt * chunks);
  for (int w = R.w; w < R.w1; w += R.step) {
    const int t = ml.list[w / chunks];
    const int c = (w % chunks) * 256 + (int)threadIdx.x;
    if (c >= nd) continue;
    const int i = c % nf + 1, row = c / nf;  // row = (k-1) nf + (j-1)
    const T* zr = ezy + (long long)t * nf * nf * nc + (long long)row * nc;
    T* o = ef + (F.voff ? F.voff[t] : (long long)t * F.ndof);
    o[c] = o[c] + prolong_x(zr, nc, ci[i - 1], cw[i - 1]);
  }
}

// dense Cholesky of each solve's coarsest operator (FP64 tables), one thread
// per solve; L (mc x mc, row-major lower) is assembled in place
__global__ void k_mg_factor(MgLv C, double* __restrict__ Lall, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C.nsol) return;
  const int n = C.n, mc = (int)C.ndof;
  double* A = Lall + (long long)t * mc * mc;
  for (int e = 0; e < mc * mc; e++) A[e] = 0.0;
  const double* kap = (const double*)C.kap + C.sd[t].kap_off;
  for (int r = 0; r < mc; r++) {
    const int i = r % n + 1, j = (r / n) % n + 1, k = r / (n * n) + 1;
    double kk[6];
    kappa6<double>(C.pd->g, kap, i, j, k, kk);
    A[r * mc + r] = diagT(kk);
    if (i > 1) A[r * mc + r - 1] = -kk[0];
    if (i < n) A[r * mc + r + 1] = -kk[1];
    if (j > 1) A[r * mc + r - n] = -kk[2];
    if (j < n) A[r * mc + r + n] = -kk[3];
    if (k > 1) A[r * mc + r - n * n] = -kk[4];
    if (k < n) A[r * mc + r + n * n] = -kk[5];
  }
  // in place: the strict upper triangle is never read again
  for (int jj = 0; jj < mc; jj++) {
    double s = A[jj * mc + jj];
    for (int kq = 0; kq < jj; kq++) s = __fma_rn(-A[jj * mc + kq], A[jj * mc + kq], s);
    if (!(s > 0.0)) {
      atomicAdd(bad, 1);
      return;
    }
    const double ljj = sqrt(s);
    A[jj * mc + jj] = ljj;
    for (int ii = jj + 1; ii < mc; ii++) {
      double u = A[ii * mc + jj];
      for (int kq = 0; kq < jj; kq++) u = __fma_rn(-A[ii * mc + kq], A[jj * mc + kq], u);
      A[ii * mc + jj] = u / ljj;
    }
  }
}

// e = A_c^{-1} b by the stored factor (FP64 arithmetic), one wave per listed
// solve.  The factor is staged in LDS; lane i holds unknown i, and the chains
// of the two triangular solves (fma over ascending k, then the division) run
// on values broadcast from the lanes that own them, in the same order as a
// sequential solve.
__device__ __forceinline__ double lane_bcast(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

template <typename T>
__global__ __launch_bounds__(64) void k_mg_coarse(MgLv C, MgList ml, const double* __restrict__ Lall,
                                                  const T* __restrict__ b, T* __restrict__ e) {
  __shared__ double Ls[27 * 27];
  if ((int)blockIdx.x >= *ml.cnt) return;  // uniform over the block
  const int lane = threadIdx.x;
  const int t = ml.list[blockIdx.x];
  const int mc = (int)C.ndof;
  const double* L = Lall + (long long)t * mc * mc;
  const long long off = C.voff ? C.voff[t] : (long long)t * C.ndof;
  for (int x = lane; x < mc * mc; x += 64) Ls[x] = L[x];
  const double bl = lane < mc ? (double)b[off + lane] : 0.0;
  __syncthreads();
  double yv = 0.0;  // y[lane]
  for (int i = 0; i < mc; i++) {
    const double Li = lane < mc ? Ls[i * mc + lane] : 0.0;  // row i: L[i][lane]
    double sacc = lane_bcast(bl, i);
    for (int k = 0; k < i; k++) sacc = __fma_rn(-lane_bcast(Li, k), lane_bcast(yv, k), sacc);
    const double yi = sacc / lane_bcast(Li, i);
    if (lane == i) yv = yi;
  }
  double xv = 0.0;  // x[lane]
  for (int i = mc - 1; i >= 0; i--) {
    const double Lc = lane < mc ? Ls[lane * mc + i] : 0.0;  // column i: L[lane][i]
    double sacc = lane_bcast(yv, i);
    for (int k = i + 1; k < mc; k++) sacc = __fma_rn(-lane_bcast(Lc, k), lane_bcast(xv, k), sacc);
    const double xi = sacc / lane_bcast(Lc, i);
    if (lane == i) xv = xi;
  }
  if (lane < mc) e[off + lane] = (T)xv;
}

// The coarsest operator's inverse from its stored factor, for the FP32 V-cycle:
// thread (t, j) solves L L^T x = e_j (forward, then backward substitution, FP64)
// and writes column j of A_c^{-1} (symmetric, stored row-major).
__global__ void k_mg_inverse(MgLv C, const double* __restrict__ Lall, double* __restrict__ Iall) {
  const int mc = (int)C.ndof;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)C.nsol * mc) return;
  const int t = (int)(idx / mc), j = (int)(idx % mc);
  const double* L = Lall + (long long)t * mc * mc;
  double* X = Iall + (long long)t * mc * mc;
  double y[27];
  for (int i = 0; i < mc; i++) {
    double sacc = i == j ? 1.0 : 0.0;
    for (int k = 0; k < i; k++) sacc = __fma_rn(-L[i * mc + k], y[k], sacc);
    y[i] = sacc / L[i * mc + i];
  }
  for (int i = mc - 1; i >= 0; i--) {
    double sacc = y[i];
    for (int k = i + 1; k < mc; k++) sacc = __fma_rn(-L[k * mc + i], y[k], sacc);
    y[i] = sacc / L[i * mc + i];  // y[k > i] now holds x[k]
  }
  for (int i = 0; i < mc; i++) X[i * mc + j] = y[i];
}

// e = A_c^{-1} b for the FP32 V-cycle, one wave per listed solve: lane i forms
// row i's dot product with b in FP64 (ascending k) and rounds it once to float.
// The sequential triangular solves of k_mg_coarse (whose order the FP64 path
// shares with the oracle) take a chain of 2 mc dependent steps with a division
// each; this is one independent chain per lane.
__global__ __launch_bounds__(64) void k_mg_coarse_inv(MgLv C, MgList ml, const double* __restrict__ Iall,
                                                      const float* __restrict__ b, float* __restrict__ e) {
  __shared__ double Is[27 * 27];
  __shared__ double bs[27];
  if ((int)blockIdx.x >= *ml.cnt) return;  // uniform over the block
  const int lane = threadIdx.x;
  const int t = ml.list[blockIdx.x];
  const int mc = (int)C.ndof;
  const double* I = Iall + (long long)t * mc * mc;
  const long long off = C.voff ? C.voff[t] : (long long)t * C.ndof;
  for (int x = lane; x < mc * mc; x += 64) Is[x] = I[x];
  if (lane < mc) bs[lane] = (double)b[off + lane];
  __syncthreads();
  if (lane < mc) {
    double acc = 0.0;
    for (int k = 0; k < mc; k++) acc = __fma_rn(Is[lane * mc + k], bs[k], acc);
    e[off + lane] = (float)acc;
  }
}

// ---------------------------------------------------------------------------
// Level 0, after the coarse correction (nu = 1): one z-march over each tile of
// the batch (the CG work items) forms e2 = e1 + P e_c at the tile's points and
// halo, keeps the current plane in LDS, and writes the post-smoothed
//   s = e2 + omega (r - A e2) / d
// with the r^T s partial of the tile (CrAcc slot 1 in FP64, IrPart.g[2] in
// FP32).  e2 never goes to memory: 12 bytes per point (FP32) instead of the 28
// of separate prolongation, smoothing and dot passes.
// ---------------------------------------------------------------------------
struct MgFine {           // per problem: the z/y-interpolated level-1 correction and transfer tables
  const void* ezy;        // group layout, t * nf * nf * nc (before it: the x-sums of the restriction)
  const int* ci;
  const void* cw;
  long long per;          // nf * nf * nc
  int nc;
  int fz;                 // 1: the FP32 post-smoothing interpolates ec itself (ezy not used)
  const int2* lohi;       // fine span of each coarse node
  const void* ec;         // the coarse correction, group layout t * nc^3
};

// LDS rings of the FP32 post-smoothing when it interpolates the coarse
// correction itself (tiles that span whole rows): three coarse planes of the
// rows the tile needs (at most kPzRing values each) and the z/y-interpolated
// rows of three fine planes (the tile's rows and its two halo rows, at most
// kPzRows values each).  The host checks both bounds per level.
constexpr int kPzRing = 448;
constexpr int kPzRows = 680;
// An ezy row in the ring: CW values behind one zero and followed by three, so
// that the four-column window of a quad and the halo point's two taps read it
// without a test for coarse columns outside the grid (they meet the zeros).
constexpr int kPzPad = 4;

// Level 0, before the coarse correction (nu = 1): e1 = omega b / d (one
// Jacobi sweep from zero) and t = b - A e1, one z-march per tile; e1 of the
// current plane and its halo (whose diagonal comes from the halo point's own
// coefficients) sit in LDS.  Only t is written (8 bytes per point in FP32
// instead of the 20 of separate smoothing and residual passes): the
// post-smoothing forms e1 again from b, with the same operations.
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_mg_pre0(const int2* __restrict__ items, const int* __restrict__ list,
                                                 const int* __restrict__ cnt, const SolveDev* __restrict__ sd,
                                                 const ProbDev* __restrict__ pd, const T* __restrict__ kap,
                                                 const T* __restrict__ b, T* __restrict__ tout, T omega,
                                                 int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  T* kt = reinterpret_cast<T*>(smem_raw);
  T* plane = kt + ktab;
  __shared__ int zk[kZkLen];
  const WorkRange WR = work_range(*cnt);
  for (int w = WR.w; w < WR.w1; w += WR.step) {
    const int item = list[w];
    __syncthreads();  // LDS of the previous item is free
    const int2 it = items[item];
    const SolveDev S = sd[it.x];
    const ProbDev& P = pd[S.prob];
    const GridDev& g = P.g;
    const int ntab = g.ndir * g.nclass;
    QuadGeo G;
    quad_geo(G, P, it.y);
    for (int e = threadIdx.x; e < ntab; e += blockDim.x) kt[e] = kap[S.kap_off + e];
    zk_stage(zk, g, G);
    __syncthreads();
    const int n = g.n, nv = G.nv;
    const long long n2 = (long long)n * n;
    const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);
    const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);
    const bool hin = G.hi != 0;
    const T* Bv = b + S.off;
    T* TO = tout + S.off;
    // raw loads of b (own quad at plane k, halo point at plane k), issued one
    // or two planes ahead of their use; e1 = omega b / d formed from them later
    auto load_b = [&](int k, T bq[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) bq[e] = T(0);
      if (nv == 0 || k < 1 || k > n) return;
      ld4<T, VEC>(Bv, (long long)(k - 1) * n2 + rowoff, nv, bq);
    };
    auto load_hb = [&](int k) __attribute__((always_inline)) -> T {
      return (!hin || k < 1 || k > n) ? T(0) : Bv[(long long)(k - 1) * n2 + hoff];
    };
    auto quad_e1 = [&](int k, const T bq[4], T out[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = T(0);
      if (nv == 0 || k < 1 || k > n) return;
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        const T dg = diag6T<T>(kk);
        T t = bq[e] - T(0);
        t = t / dg;
        out[e] = in_quad<VEC>(e, nv) ? fmaT(omega, t, T(0)) : T(0);
      }
    };
    auto halo_e1 = [&](int k, T braw) __attribute__((always_inline)) -> T {
      if (!hin || k < 1 || k > n) return T(0);
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
      T kk[6];
      kk[0] = kt[G.hb[0] + czn];
      kk[1] = kt[G.hb[1] + czn];
      kk[2] = kt[G.hb[2] + czn];
      kk[3] = kt[G.hb[3] + czn];
      kk[4] = kt[G.hb[4] + czm];
      kk[5] = kt[G.hb[4] + czp];
      const T dg = diag6T<T>(kk);
      T t = braw - T(0);
      t = t / dg;
      return fmaT(omega, t, T(0));
    };
    T um[4], uc[4], un[4], bm[4], bc[4], bn[4], bnn[4];
    load_b(G.kb - 1, bm);
    load_b(G.kb, bc);
    load_b(G.kb + 1, bn);
    T hbc = load_hb(G.kb);
    quad_e1(G.kb - 1, bm, um);
    quad_e1(G.kb, bc, uc);
    int buf = 0;
    const int mrow = G.mrow;

    for (int k = G.kb; k <= G.ke; k++) {
      load_b(k + 2, bnn);
      const T hbn = load_hb(k + 1);
      quad_e1(k + 1, bn, un);
      const T hv = halo_e1(k, hbc);
      T* pl = plane + buf * QPLANE;
      pl_st4(pl + mrow, uc);
      if (G.hslot >= 0) pl[G.hslot] = hv;
      __syncthreads();
      T left, right;
      quad_xnb<T>(G, pl, uc, left, right);
      if (nv > 0) {
        const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
        const long long c = (long long)(k - 1) * n2 + rowoff;
        T ymv[4], ypv[4];
        pl_ld4(pl + mrow - G.qs, ymv);
        pl_ld4(pl + mrow + G.qs, ypv);
        T to[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          T kk[6];
          quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
          const T dg = diag6T<T>(kk);
          T q = dg * uc[e];
          q = fmaT(-kk[0], e > 0 ? uc[e - 1] : left, q);
          q = fmaT(-kk[1], e < 3 ? uc[e + 1] : right, q);
          q = fmaT(-kk[2], ymv[e], q);
          q = fmaT(-kk[3], ypv[e], q);
          q = fmaT(-kk[4], um[e], q);
          q = fmaT(-kk[5], un[e], q);
          to[e] = bc[e] - q;
        }
        st4<T, VEC>(TO, c, nv, to);
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        um[e] = uc[e];
        uc[e] = un[e];
        bc[e] = bn[e];
        bn[e] = bnn[e];
      }
      hbc = hbn;
      buf ^= 1;
    }
  }
}

template <typename T> struct PostPart;
template <> struct PostPart<double> {
  static __device__ __forceinline__ void put(void* part, int item, DotAcc<double>& a, CrAcc* red) {
    const CrAcc t = cr_block_reduce(a.a, red);
    if (threadIdx.x == 0) ((CrAcc*)part)[(long long)item * kSlots + 1] = t;
  }
};
template <> struct PostPart<float> {
  static __device__ __forceinline__ void put(void* part, int item, DotAcc<float>& a, CrAcc* red) {
    double g = a.a;
    for (int m = 32; m >= 1; m >>= 1) g += __shfl_xor(g, m, 64);
    double* rd = reinterpret_cast<double*>(red);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) rd[threadIdx.x >> 6] = g;
    __syncthreads();
    if (threadIdx.x == 0) ((IrPart*)part)[item].g[2] = rd[0] + rd[1] + rd[2] + rd[3];
  }
};

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_mg_post0(const int2* __restrict__ items, const int* __restrict__ list,
                                                  const int* __restrict__ cnt, const SolveDev* __restrict__ sd,
                                                  const ProbDev* __restrict__ pd, const T* __restrict__ kap,
                                                  const MgFine* __restrict__ mf, const int* __restrict__ gidx,
                                                  const T* __restrict__ r, T* __restrict__ sout, void* part,
                                                  T omega, int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  T* kt = reinterpret_cast<T*>(smem_raw);
  T* plane = kt + ktab;
  __shared__ CrAcc red[4];
  __shared__ int zk[kZkLen];
  const WorkRange WR = work_range(*cnt);
  for (int w = WR.w; w < WR.w1; w += WR.step) {
    const int item = list[w];
    __syncthreads();  // LDS of the previous item is free
    const int2 it = items[item];
    const int b = it.x;
    const SolveDev S = sd[b];
    const ProbDev& P = pd[S.prob];
    const GridDev& g = P.g;
    const MgFine F = mf[S.prob];
    const gptr<T> ezy = as_global((const T*)F.ezy) + (long long)gidx[b] * F.per;
    const gptr<T> cw = as_global((const T*)F.cw);
    const int ntab = g.ndir * g.nclass;
    QuadGeo G;
    quad_geo(G, P, it.y);
    for (int e = threadIdx.x; e < ntab; e += blockDim.x) kt[e] = kap[S.kap_off + e];
    zk_stage(zk, g, G);
    __syncthreads();
    const int n = g.n, nv = G.nv;
    const long long n2 = (long long)n * n;
    const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);
    const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);
    const bool hin = G.hi != 0;
    const T* R = r + S.off;
    T* SO = sout + S.off;
    // transfer weights of the quad's x points, its row and the halo point
    int I0[4];
    T wx[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int i = min(G.i + e, n);
      I0[e] = F.ci[i - 1];
      wx[e] = cw[i - 1];
    }
    const int nc = F.nc;
    const int jj = min(G.j, n);
    const int hI0 = hin ? F.ci[G.hi - 1] : 0;
    const T hwx = hin ? cw[G.hi - 1] : T(0);
    // raw loads (r and the two x taps of ezy) for the own quad and the halo
    // point, issued ahead of their use; then e2 = e1 + P_x ezy with e1 the
    // pre-smoothing omega r / d, formed as the pre-smoothing forms it
    auto taps = [&](gptr<T> zr, int i0, T& za, T& zb) __attribute__((always_inline)) {
      za = i0 >= 1 ? zr[i0 - 1] : T(0);
      zb = i0 + 1 <= nc ? zr[i0] : T(0);
    };
    auto join = [&](int i0, T w, T za, T zb) __attribute__((always_inline)) -> T {
      T v = T(0);
      if (i0 >= 1) v = fmaT(T(1) - w, za, v);
      if (i0 + 1 <= nc) v = fmaT(w, zb, v);
      return v;
    };
    auto jac = [&](T rv, T dg) __attribute__((always_inline)) -> T {
      T t = rv - T(0);
      t = t / dg;
      return fmaT(omega, t, T(0));
    };
    struct Raw {
      T r[4], za[4], zb[4];
    };
    auto load_q = [&](int k, Raw& q) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) q.r[e] = q.za[e] = q.zb[e] = T(0);
      if (nv == 0 || k < 1 || k > n) return;
      ld4<T, VEC>(R, (long long)(k - 1) * n2 + rowoff, nv, q.r);
      const gptr<T> zr = ezy + ((long long)(k - 1) * n + (jj - 1)) * nc;
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (in_quad<VEC>(e, nv)) taps(zr, I0[e], q.za[e], q.zb[e]);
    };
    auto fin_q = [&](int k, const Raw& q, T out[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = T(0);
      if (nv == 0 || k < 1 || k > n) return;
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        T kk[6];
        quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
        const T dg = diag6T<T>(kk);
        out[e] = in_quad<VEC>(e, nv) ? jac(q.r[e], dg) + join(I0[e], wx[e], q.za[e], q.zb[e]) : T(0);
      }
    };
    struct RawH {
      T r, za, zb;
    };
    auto load_h = [&](int k, RawH& h) __attribute__((always_inline)) {
      h.r = h.za = h.zb = T(0);
      if (!hin || k < 1 || k > n) return;
      h.r = R[(long long)(k - 1) * n2 + hoff];
      taps(ezy + ((long long)(k - 1) * n + (G.hj - 1)) * nc, hI0, h.za, h.zb);
    };
    auto fin_h = [&](int k, const RawH& h) __attribute__((always_inline)) -> T {
      if (!hin || k < 1 || k > n) return T(0);
      const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
      T kk[6];
      kk[0] = kt[G.hb[0] + czn];
      kk[1] = kt[G.hb[1] + czn];
      kk[2] = kt[G.hb[2] + czn];
      kk[3] = kt[G.hb[3] + czn];
      kk[4] = kt[G.hb[4] + czm];
      kk[5] = kt[G.hb[4] + czp];
      const T dg = diag6T<T>(kk);
      return jac(h.r, dg) + join(hI0, hwx, h.za, h.zb);
    };
    T um[4], uc[4], un[4], rc[4];
    Raw qn, qnn;
    {
      Raw qm, qc;
      load_q(G.kb - 1, qm);
      load_q(G.kb, qc);
      load_q(G.kb + 1, qn);
      fin_q(G.kb - 1, qm, um);
      fin_q(G.kb, qc, uc);
#pragma unroll
      for (int e = 0; e < 4; e++) rc[e] = qc.r[e];
    }
    RawH hc;
    load_h(G.kb, hc);
    DotAcc<T> acc;
    acc.zero();
    int buf = 0;
    const int mrow = G.mrow;

    for (int k = G.kb; k <= G.ke; k++) {
      load_q(k + 2, qnn);
      RawH hn;
      load_h(k + 1, hn);
      fin_q(k + 1, qn, un);
      const T hv = fin_h(k, hc);
      T* pl = plane + buf * QPLANE;
      pl_st4(pl + mrow, uc);
      if (G.hslot >= 0) pl[G.hslot] = hv;
      __syncthreads();
      T left, right;
      quad_xnb<T>(G, pl, uc, left, right);
      if (nv > 0) {
        const int zkv = G.zk[k - G.kb + 1], czn = zkv & 255, czm = (zkv >> 8) & 255, czp = zkv >> 16;
        const long long c = (long long)(k - 1) * n2 + rowoff;
        T ymv[4], ypv[4];
        pl_ld4(pl + mrow - G.qs, ymv);
        pl_ld4(pl + mrow + G.qs, ypv);
        T so[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          T kk[6];
          quad_kappa<T>(G, kt, e, czn, czm, czp, kk);
          const T dg = diag6T<T>(kk);
          T q = dg * uc[e];
          q = fmaT(-kk[0], e > 0 ? uc[e - 1] : left, q);
          q = fmaT(-kk[1], e < 3 ? uc[e + 1] : right, q);
          q = fmaT(-kk[2], ymv[e], q);
          q = fmaT(-kk[3], ypv[e], q);
          q = fmaT(-kk[4], um[e], q);
          q = fmaT(-kk[5], un[e], q);
          T t = rc[e] - q;
          t = t / dg;
          so[e] = fmaT(omega, t, uc[e]);
          if (in_quad<VEC>(e, nv)) acc.add(rc[e], so[e]);
        }
        st4<T, VEC>(SO, c, nv, so);
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        um[e] = uc[e];
        uc[e] = un[e];
        rc[e] = qn.r[e];
      }
      qn = qnn;
      hc = hn;
      buf ^= 1;
    }
    PostPart<T>::put(part, item, acc, red);
  }
}

// FP32 fused smoothing kernels of a level (nu = 1), tile z-marches like the
// FP64 ones above.  The own quad's face coefficients, diagonal and reciprocal
// diagonal, and the halo point's reciprocal diagonal, sit in registers
// (KCache32, refreshed only when the plane's z codes change), so a plane costs
// no class-table reads and no division: Jacobi is omega (r (1/d)).  e1 of plane
// k+1, needed by the stencil of plane k, takes its reciprocals from a second
// cache keyed by plane k+1.  The pre- and post-smoothing form e1 with the same
// operations.  Items: with ML false, the tiles on a work list (level 0, the
// CG's list of the listed solves); with ML true, every tile of the solves on a
// V-cycle list (item = list[w / ntiles] * ntiles + w % ntiles, levels >= 1,
// whose batches hold ntiles tiles per solve, solve-major).
struct InvCache32 {
  int key;
  float inv[4];
};
__device__ __forceinline__ void inv_fill(InvCache32& C, const QuadGeo& G, const float* kt, int key) {
  const int czn = key & 255, czm = (key >> 8) & 255, czp = key >> 16;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    float kk[6];
    quad_kappa<float>(G, kt, e, czn, czm, czp, kk);
    C.inv[e] = 1.0f / diag6T<float>(kk);
  }
  C.key = key;
}

// shared set-up of an item of the FP32 level-0 kernels
#define MG0_ITEM_SETUP()                                                                \
  const int item = ML ? list[w / ntiles] * ntiles + w % ntiles : list[w];              \
  __syncthreads(); /* LDS of the previous item is free */                               \
  const int2 it = items[item];                                                          \
  const SolveDev S = sd[it.x];                                                          \
  const ProbDev& P = pd[S.prob];                                                        \
  const GridDev& g = P.g;                                                               \
  const int ntab = g.ndir * g.nclass;                                                   \
  QuadGeo G;                                                                            \
  quad_geo(G, P, it.y);                                                                 \
  for (int e = threadIdx.x; e < ntab; e += blockDim.x) kt[e] = kap[S.kap_off + e];      \
  zk_stage(zk, g, G);                                                                   \
  __syncthreads();                                                                      \
  const int n = g.n, nv = G.nv;                                                         \
  const long long n2 = (long long)n * n;                                                \
  const long long rowoff = ((long long)(G.j - 1)) * n + (G.i - 1);                      \
  const long long hoff = ((long long)(G.hj - 1)) * n + (G.hi - 1);                      \
  const bool hin = G.hi != 0;                                                           \
  const int mrow = G.mrow;                                          \
  \
  auto zkey_at = [&](int k) __attribute__((always_inline)) { return G.zk[k - G.kb + 1]; };

// q = A u at the own quad of plane k (u of plane k in registers and LDS; the
// planes k-1, k+1 in um, un), coefficients from the cache
#define MG0_STENCIL(C, um, uc, un, pl, left, right, q)                                  \
  {                                                                                     \
    float ymv[4], ypv[4];                                                               \
    pl_ld4(pl + mrow - G.qs, ymv);                                                      \
    pl_ld4(pl + mrow + G.qs, ypv);                                                      \
    _Pragma("unroll") for (int e = 0; e < 4; e++) {                                     \
      float a = C.dg[e] * uc[e];                                                        \
      a = fmaf(-C.kx[e], e > 0 ? uc[e - 1] : left, a);                                  \
      a = fmaf(-C.kx[e + 1], e < 3 ? uc[e + 1] : right, a);                             \
      a = fmaf(-C.kym[e], ymv[e], a);                                                   \
      a = fmaf(-C.kyp[e], ypv[e], a);                                                   \
      a = fmaf(-C.kzm[e], um[e], a);                                                    \
      a = fmaf(-C.kzp[e], un[e], a);                                                    \
      q[e] = a;                                                                         \
    }                                                                                   \
  }

// The post-smoothing keeps fewer registers (four waves per SIMD instead of
// three): only d, 1/d and the z codes are cached; the face coefficients of
// the stencil come from the class table in LDS.  The values are the same.
struct DCache32 {
  int key, czn, czm, czp;
  float dg[4], inv[4];
  float hinv;
};
__device__ __forceinline__ void dc_fill(DCache32& C, const QuadGeo& G, const float* kt, int key) {
  C.czn = key & 255;
  C.czm = (key >> 8) & 255;
  C.czp = key >> 16;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    float kk[6];
    quad_kappa<float>(G, kt, e, C.czn, C.czm, C.czp, kk);
    C.dg[e] = diag6T<float>(kk);
    C.inv[e] = 1.0f / C.dg[e];
  }
  C.hinv = 1.0f;
  if (G.hi != 0) {
    const float hd = ((((kt[G.hb[0] + C.czn] + kt[G.hb[1] + C.czn]) + kt[G.hb[2] + C.czn]) + kt[G.hb[3] + C.czn]) +
                      kt[G.hb[4] + C.czm]) +
                     kt[G.hb[4] + C.czp];
    C.hinv = 1.0f / hd;
  }
  C.key = key;
}
#define MG0_STENCIL_LDS(C, um, uc, un, pl, left, right, q)                              \
  {                                                                                     \
    float ymv[4], ypv[4];                                                               \
    pl_ld4(pl + mrow - G.qs, ymv);                                                      \
    pl_ld4(pl + mrow + G.qs, ypv);                                                      \
    _Pragma("unroll") for (int e = 0; e < 4; e++) {                                     \
      float kk[6];                                                                      \
      quad_kappa<float>(G, kt, e, C.czn, C.czm, C.czp, kk);                             \
      float a = C.dg[e] * uc[e];                                                        \
      a = fmaf(-kk[0], e > 0 ? uc[e - 1] : left, a);                                    \
      a = fmaf(-kk[1], e < 3 ? uc[e + 1] : right, a);                                   \
      a = fmaf(-kk[2], ymv[e], a);                                                      \
      a = fmaf(-kk[3], ypv[e], a);                                                      \
      a = fmaf(-kk[4], um[e], a);                                                       \
      a = fmaf(-kk[5], un[e], a);                                                       \
      q[e] = a;                                                                         \
    }                                                                                   \
  }

// With RX (tiles that span the whole row) the residual t is not written:
// each fine row of it goes through LDS and the kernel writes the restriction's
// x-sums ax[k][j][I] = sum_i px t (fma chain from 0, ascending i) into the
// level's MgFine buffer, n_c values per row instead of n.  The rows in LDS
// have a stride of TX + 4 floats (16-byte aligned: a quad goes in with one
// 16-byte store; an odd stride would put the two rows a wave covers on
// different banks for the x-sum reads but needs four scalar stores at two-way
// conflicts, which measured slower) and are zeroed per item: every chain takes
// all kSpan taps, those past the node's span with weight 0 on a finite value,
// which leaves the chain's value unchanged, without a branch per tap.
constexpr int kTrow = 1280;  // floats per LDS plane of t: rows x (TX + 4) <= 1152 (TX >= 32)
template <bool VEC, bool ML, bool RX>
__global__ __launch_bounds__(256, 4) void k_mg_pre0_32(const int2* __restrict__ items, const int* __restrict__ list,
                                                    const int* __restrict__ cnt, int ntiles,
                                                    const SolveDev* __restrict__ sd,
                                                    const ProbDev* __restrict__ pd, const float* __restrict__ kap,
                                                    const float* __restrict__ b, float* __restrict__ tout,
                                                    const MgFine* __restrict__ mf, const int* __restrict__ gidx,
                                                    float omega, int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  float* kt = reinterpret_cast<float*>(smem_raw);
  float* plane = kt + ktab;
  __shared__ int zk[kZkLen];
  __shared__ __align__(16) float trow[RX ? 2 * kTrow + 8 : 1];  // the tile's t of two planes
  __shared__ float xw[RX ? 64 : 1][kSpan];       // x weights per coarse column
  __shared__ int xlo[RX ? 64 : 1];
  const WorkRange WR = work_range(ML ? *cnt * ntiles : *cnt);
  for (int w = WR.w; w < WR.w1; w += WR.step) {
    MG0_ITEM_SETUP()
    const float* Bv = b + S.off;
    float* TO = tout + S.off;
    float* txo = nullptr;
    int nc = 0;
    const int txw = 4 * (G.lxm + 1) + 4;  // row stride of trow (the tile spans the row)
    if constexpr (RX) {
      const MgFine F = mf[S.prob];
      nc = F.nc;
      txo = (float*)F.ezy + (long long)(ML ? it.x : gidx[it.x]) * F.per;
      const float* cw = (const float*)F.cw;
      for (int I = threadIdx.x + 1; I <= nc; I += blockDim.x) {
        const int2 r = F.lohi[I];
        xlo[I - 1] = r.x;
#pragma unroll
        for (int u = 0; u < kSpan; u++) {
          const int i = r.x + u;
          xw[I - 1][u] = i <= r.y ? (F.ci[i - 1] == I ? 1.0f - cw[i - 1] : cw[i - 1]) : 0.0f;
        }
      }
      for (int e = threadIdx.x; e < 2 * kTrow + 8; e += blockDim.x) trow[e] = 0.0f;
      __syncthreads();
    }
    auto load_b = [&](int k, float bq[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) bq[e] = 0.0f;
      if (nv == 0 || k < 1 || k > n) return;
      ld4<float, VEC>(Bv, (long long)(k - 1) * n2 + rowoff, nv, bq);
    };
    auto load_hb = [&](int k) __attribute__((always_inline)) -> float {
      return (!hin || k < 1 || k > n) ? 0.0f : Bv[(long long)(k - 1) * n2 + hoff];
    };
    KCache32 C;
    InvCache32 Ci;
    C.key = Ci.key = -1;
    auto e1_quad = [&](int k, const float bq[4], float out[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = 0.0f;
      if (nv == 0 || k < 1 || k > n) return;
      const int key = zkey_at(k);
      if (key != Ci.key) inv_fill(Ci, G, kt, key);
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = in_quad<VEC>(e, nv) ? omega * (bq[e] * Ci.inv[e]) : 0.0f;
    };
    // x-sums of plane k's rows from trow (buffer tb); the writes of that plane
    // are ordered before these reads by the next plane's barrier
    // (a thread has at most two coarse columns: n_c <= (n - 1) / 2 < 2 (lxm + 1))
    auto xsums = [&](int k, int tb) __attribute__((always_inline)) {
      if constexpr (RX) {
        if (G.j <= n) {
          const gptr_w<float> o = as_global_w(txo) + ((long long)(k - 1) * n + (G.j - 1)) * nc;
          const float* tr = trow + tb * kTrow + G.ly * txw - 1;
#pragma unroll
          for (int m = 0; m < 2; m++) {
            const int I = G.lx + 1 + m * (G.lxm + 1);
            if (I > nc) break;
            const float* t = tr + xlo[I - 1];
            float ax = 0.0f;
#pragma unroll
            for (int u = 0; u < kSpan; u++) ax = fmaf(xw[I - 1][u], t[u], ax);
            o[I - 1] = ax;
          }
        }
      }
    };
    float um[4], uc[4], un[4], bm[4], bc[4], bn[4], bnn[4];
    load_b(G.kb - 1, bm);
    load_b(G.kb, bc);
    load_b(G.kb + 1, bn);
    float hbc = load_hb(G.kb);
    e1_quad(G.kb - 1, bm, um);
    e1_quad(G.kb, bc, uc);
    int buf = 0;
    for (int k = G.kb; k <= G.ke; k++) {
      load_b(k + 2, bnn);
      const float hbn = load_hb(k + 1);
      const int key = zkey_at(k);
      if (key != C.key) kc_fill(C, G, kt, key);
      e1_quad(k + 1, bn, un);
      float* pl = plane + buf * QPLANE;
      pl_st4(pl + mrow, uc);
      if (G.hslot >= 0) pl[G.hslot] = hin ? omega * (hbc * C.hinv) : 0.0f;
      __syncthreads();
      if (k > G.kb) xsums(k - 1, buf ^ 1);
      float left, right;
      quad_xnb<float>(G, pl, uc, left, right);
      if (nv > 0) {
        float q[4], to[4];
        MG0_STENCIL(C, um, uc, un, pl, left, right, q)
#pragma unroll
        for (int e = 0; e < 4; e++) to[e] = bc[e] - q[e];
        if constexpr (RX) {
          if constexpr (VEC) {
            pl_st4(trow + buf * kTrow + G.ly * txw + 4 * G.lx, to);
          } else {
#pragma unroll
            for (int e = 0; e < 4; e++)
              if (in_quad<VEC>(e, nv)) trow[buf * kTrow + G.ly * txw + 4 * G.lx + e] = to[e];
          }
        } else {
          st4<float, VEC>(TO, (long long)(k - 1) * n2 + rowoff, nv, to);
        }
      }

#pragma unroll
      for (int e = 0; e < 4; e++) {
        um[e] = uc[e];
        uc[e] = un[e];
        bc[e] = bn[e];
        bn[e] = bnn[e];
      }
      hbc = hbn;
      buf ^= 1;
    }
    if constexpr (RX) {
      __syncthreads();
      xsums(G.ke, buf ^ 1);
    }
  }
}

// With PZ (tiles that span whole rows) the kernel also does the z/y
// interpolation of the coarse correction: per tile it stages the coarse planes
// it needs in an LDS ring and forms ezy of plane k+2 while plane k is smoothed,
// with the operations of k_mg_pyz, so ezy never goes to memory.
template <bool VEC, bool ML, bool PZ>
__global__ __launch_bounds__(256, 4) void k_mg_post0_32(const int2* __restrict__ items, const int* __restrict__ list,
                                                     const int* __restrict__ cnt, int ntiles,
                                                     const SolveDev* __restrict__ sd,
                                                     const ProbDev* __restrict__ pd, const float* __restrict__ kap,
                                                     const MgFine* __restrict__ mf, const int* __restrict__ gidx,
                                                     const float* __restrict__ r, float* __restrict__ sout,
                                                     IrPart* __restrict__ part, float omega, int ktab) {
  extern __shared__ __align__(16) double smem_raw[];
  float* kt = reinterpret_cast<float*>(smem_raw);
  float* plane = kt + ktab;
  __shared__ double red[4];
  __shared__ int zk[kZkLen];
  __shared__ float cring[PZ ? 3 * kPzRing : 1];  // coarse planes K at slot K % 3
  __shared__ float zring[PZ ? 3 * kPzRows : 1];  // ezy of fine plane k at slot k % 3
  __shared__ int zrow[PZ ? 40 : 1];              // per ezy row: ring offset of row J0 and flags, or -1
  __shared__ float zwy[PZ ? 40 : 1];             // per ezy row: the y weight
  __shared__ int zK[PZ ? kZkLen + 2 : 1];        // ci(kk) of the planes kb-1 .. ke+4 (index kk - kb + 1)
  __shared__ float zW[PZ ? kZkLen + 2 : 1];      // the z weight of the same planes
  const WorkRange WR = work_range(ML ? *cnt * ntiles : *cnt);
  for (int w = WR.w; w < WR.w1; w += WR.step) {
    MG0_ITEM_SETUP()
    const MgFine F = mf[S.prob];
    const gptr<float> ezy = as_global((const float*)F.ezy) + (long long)(ML ? it.x : gidx[it.x]) * F.per;
    const gptr<float> cw = as_global((const float*)F.cw);
    const float* R = r + S.off;
    float* SO = sout + S.off;
    // the quad's x points take their two coarse taps from the window of four
    // coarse columns W0 .. W0+3 (W0 = I0 of the first point, minus one): with
    // (nc+1)/(nf+1) <= 1/2, I0 grows by at most 2 over the quad.  Point e
    // weighs column I0 - 1 - W0 by 1 - w and the next by w (a coarse node
    // outside the grid by 0) and the others by 0; the weighted sum runs over
    // the window in ascending order, so the two taps enter in the order of
    // the separate pass (zero terms add nothing)
    float xw[4][4];
    const int nc = F.nc;
    const int W0 = F.ci[min(G.i, n) - 1] - 1;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int i = min(G.i + e, n);
      const int I0 = F.ci[i - 1];
      const int d = I0 - 1 - W0;
      const float w = cw[i - 1];
#pragma unroll
      for (int m = 0; m < 4; m++)
        xw[e][m] = (m == d && I0 >= 1) ? 1.0f - w : ((m == d + 1 && I0 + 1 <= nc) ? w : 0.0f);
    }
    bool wv[4];
#pragma unroll
    for (int m = 0; m < 4; m++) wv[m] = W0 + m >= 0 && W0 + m < nc;
    const int jj = min(G.j, n);
    const int hI0 = hin ? F.ci[G.hi - 1] : 0;
    const float hwx = hin ? cw[G.hi - 1] : 0.0f;
    // PZ: ezy rows j0-1 .. j0+TY of a plane (row zr = j - j0 + 1, CW values
    // each) and coarse rows Jb .. Jb+CR-1 of a plane, CW values each
    const int j0 = G.j - G.ly;
    const int CW = nc <= 16 ? 16 : nc <= 32 ? 32 : 64;
    const int cws = CW == 16 ? 4 : CW == 32 ? 5 : 6;
    const int nz = (P.TY + 2) << cws;
    const int Jb = F.ci[max(j0 - 1, 1) - 1];
    const int ncr = (F.ci[min(j0 + P.TY, n) - 1] + 2 - Jb) << cws;
    const gptr<float> ecs =
        as_global((const float*)F.ec) + (long long)(ML ? it.x : gidx[it.x]) * ((long long)nc * nc * nc);
    // ezy row zr (fine row j = j0 - 1 + zr): ring offset of coarse row J0 = ci(j)
    // (rows outside the grid: offset 0, never read) and the y weight; read after
    // the prologue's first barrier
    if constexpr (PZ) {
      const int zr = threadIdx.x, j = j0 - 1 + zr;
      if (zr < P.TY + 2) {
        const bool in = j >= 1 && j <= n;
        zrow[zr] = in ? (F.ci[j - 1] - Jb) << cws : 0;
        zwy[zr] = in ? cw[j - 1] : 0.0f;
      }
    }
    // coarse plane K of the tile's rows (zero outside the coarse grid); the
    // thread's two ring entries and their offsets within a coarse plane are
    // the same for every K
    int coff[2];
#pragma unroll
    for (int m = 0; m < 2; m++) {
      const int e = (int)threadIdx.x + 256 * m;
      const int J = Jb + (e >> cws), I = (e & (CW - 1)) + 1;
      coff[m] = (e < ncr && J >= 1 && J <= nc && I <= nc) ? (J - 1) * nc + (I - 1) : -1;
    }
    auto cload = [&](int K, float v[2]) __attribute__((always_inline)) {
      const bool kin = K >= 1 && K <= nc;
      const gptr<float> pk = ecs + (long long)(kin ? K - 1 : 0) * nc * nc;
#pragma unroll
      for (int m = 0; m < 2; m++) v[m] = (kin && coff[m] >= 0) ? pk[coff[m]] : 0.0f;
    };
    auto cstore = [&](int K, const float v[2]) __attribute__((always_inline)) {
      float* D = cring + (K % 3) * kPzRing;
#pragma unroll
      for (int m = 0; m < 2; m++) {
        const int e = (int)threadIdx.x + 256 * m;
        if (e < ncr) D[e] = v[m];
      }
    };
    // ezy of fine plane kk into its slot.  The ring holds zeros for coarse
    // nodes outside the grid, so every tap is taken: a zero tap adds an exact
    // zero, and the values are those of k_mg_pyz, which skips such taps.
    // the thread's ezy entries e = tid + 256 q (at most three: nz <= 640), their
    // ring offsets within a coarse plane and their y weights, the same for
    // every plane (set after the prologue's first barrier)
    int zo[3];
    float zy[3];
    // ring position of entry e = tid + 256 q: e + kPzPad (e >> cws) + 1, with
    // e >> cws = (tid >> cws) + q (256 >> cws) since CW divides 256
    const int zd0 = (int)threadIdx.x + kPzPad * ((int)threadIdx.x >> cws) + 1;
    const int zdq = 256 + kPzPad * (256 >> cws);
    const int zrs = CW + kPzPad;  // ring row stride
    auto zplane = [&](int kk) __attribute__((always_inline)) {
      if (kk < 1 || kk > n) return;
      float* Z = zring + (kk % 3) * kPzRows;
      const int K0 = zK[kk - G.kb + 1];
      const float wz1 = zW[kk - G.kb + 1], wz0 = 1.0f - wz1;
      const float* A = cring + (K0 % 3) * kPzRing;
      const float* Bq = cring + ((K0 + 1) % 3) * kPzRing;
#pragma unroll
      for (int q = 0; q < 3; q++) {
        if (zo[q] < 0) continue;
        const int o = zo[q];
        const float wy1 = zy[q];
        const float az0 = fmaf(wz1, Bq[o], wz0 * A[o]);
        const float az1 = fmaf(wz1, Bq[o + CW], wz0 * A[o + CW]);
        Z[zd0 + zdq * q] = fmaf(wy1, az1, (1.0f - wy1) * az0);
      }
    };
    // the upper coarse plane that ezy of fine plane kk needs (from memory in
    // the prologue, from the staged zK in the march)
    auto ptop = [&](int kk) __attribute__((always_inline)) { return F.ci[min(kk, n) - 1] + 1; };
    auto ptopL = [&](int kk) __attribute__((always_inline)) { return zK[kk - G.kb + 1] + 1; };
    auto taps = [&](gptr<float> zr, int i0, float& za, float& zb) __attribute__((always_inline)) {
      za = i0 >= 1 ? zr[i0 - 1] : 0.0f;
      zb = i0 + 1 <= nc ? zr[i0] : 0.0f;
    };
    auto join = [&](int i0, float wgt, float za, float zb) __attribute__((always_inline)) -> float {
      float v = 0.0f;
      if (i0 >= 1) v = fmaf(1.0f - wgt, za, v);
      if (i0 + 1 <= nc) v = fmaf(wgt, zb, v);
      return v;
    };

    struct Raw {
      float r[4], z[4];
    };
    auto load_q = [&](int k, Raw& q) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) q.r[e] = q.z[e] = 0.0f;
      if (nv == 0 || k < 1 || k > n) return;
      ld4<float, VEC>(R, (long long)(k - 1) * n2 + rowoff, nv, q.r);
      if constexpr (!PZ) {
        const gptr<float> zr = ezy + ((long long)(k - 1) * n + (jj - 1)) * nc + W0;
#pragma unroll
        for (int m = 0; m < 4; m++)
          if (wv[m]) q.z[m] = zr[m];
      }
    };

    struct RawH {
      float r, za, zb;
    };
    auto load_h = [&](int k, RawH& h) __attribute__((always_inline)) {
      h.r = h.za = h.zb = 0.0f;
      if (!hin || k < 1 || k > n) return;
      h.r = R[(long long)(k - 1) * n2 + hoff];
      if constexpr (!PZ) taps(ezy + ((long long)(k - 1) * n + (G.hj - 1)) * nc, hI0, h.za, h.zb);
    };
    DCache32 C;
    InvCache32 Ci;
    C.key = Ci.key = -1;
    // e2 = e1 + P_x ezy of the own quad at plane k (e1 = omega r (1/d))
    auto e2_quad = [&](int k, const Raw& q, float out[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int e = 0; e < 4; e++) out[e] = 0.0f;
      if (nv == 0 || k < 1 || k > n) return;
      const int key = zkey_at(k);
      if (key != Ci.key) inv_fill(Ci, G, kt, key);
      float z[4];
#pragma unroll
      for (int m = 0; m < 4; m++) z[m] = q.z[m];
      if constexpr (PZ) {
        const float* Zr = zring + (k % 3) * kPzRows + (jj - j0 + 1) * zrs + 1 + W0;
#pragma unroll
        for (int m = 0; m < 4; m++) z[m] = Zr[m];
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        float v = xw[e][0] * z[0];
        v = fmaf(xw[e][1], z[1], v);
        v = fmaf(xw[e][2], z[2], v);
        v = fmaf(xw[e][3], z[3], v);
        out[e] = in_quad<VEC>(e, nv) ? omega * (q.r[e] * Ci.inv[e]) + v : 0.0f;
      }
    };
    float pf[2] = {0.0f, 0.0f};  // PZ: the next coarse plane, loaded one iteration ahead
    int Pcur = 0, Pnext = 0;
    if constexpr (PZ) {
      // ci and the z weight of the planes kb-1 .. ke+4 (clamped to the grid)
      for (int t = threadIdx.x; t < G.ke - G.kb + 6; t += 256) {
        const int kc = min(max(G.kb - 1 + t, 1), n);
        zK[t] = F.ci[kc - 1];
        zW[t] = cw[kc - 1];
      }
      for (int t = threadIdx.x; t < 3 * kPzRows; t += 256) zring[t] = 0.0f;  // the rows' zero pads
      // ezy of planes kb-1 .. kb+1 (coarse planes ci(kb-1) .. ci(kb+1)+1, at most three)
      const int Ka = F.ci[max(G.kb - 1, 1) - 1], Kz = ptop(G.kb + 1);
      for (int K = Ka; K <= Kz; K++) {
        float v[2];
        cload(K, v);
        cstore(K, v);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int e = (int)threadIdx.x + 256 * q;
        zo[q] = -1;
        zy[q] = 0.0f;
        if (e < nz) {
          zo[q] = zrow[e >> cws] + (e & (CW - 1));
          zy[q] = zwy[e >> cws];
        }
      }
      zplane(G.kb - 1);
      zplane(G.kb);
      zplane(G.kb + 1);
      __syncthreads();
      // the loop's ring: planes Pcur-1 and Pcur (ezy of plane kb+2), the next one prefetched
      Pcur = ptop(G.kb + 2);
      Pnext = ptop(G.kb + 3);
      {
        float v[2];
        cload(Pcur - 1, v);
        cstore(Pcur - 1, v);
        cload(Pcur, v);
        cstore(Pcur, v);
      }
      if (Pnext != Pcur) cload(Pnext, pf);
      __syncthreads();
    }
    float um[4], uc[4], un[4], rc[4];
    Raw qn, qnn;
    {
      Raw qm, qc;
      load_q(G.kb - 1, qm);
      load_q(G.kb, qc);
      load_q(G.kb + 1, qn);
      e2_quad(G.kb - 1, qm, um);
      e2_quad(G.kb, qc, uc);
#pragma unroll
      for (int e = 0; e < 4; e++) rc[e] = qc.r[e];
    }
    // the first iteration writes the z ring slot that e2_quad(kb - 1) read
    if constexpr (PZ) __syncthreads();
    RawH hc;
    load_h(G.kb, hc);
    double acc = 0.0;
    int buf = 0;
    for (int k = G.kb; k <= G.ke; k++) {
      load_q(k + 2, qnn);
      RawH hn;
      load_h(k + 1, hn);
      const int key = zkey_at(k);
      if (key != C.key) dc_fill(C, G, kt, key);
      e2_quad(k + 1, qn, un);
      float* pl = plane + buf * QPLANE;
      pl_st4(pl + mrow, uc);
      if constexpr (PZ) {
        if (hin) {
          const float* Zh = zring + (k % 3) * kPzRows + (G.hj - j0 + 1) * zrs + 1;
          hc.za = Zh[hI0 - 1];
          hc.zb = Zh[hI0];
        }
      }
      if (G.hslot >= 0) {
        // with PZ the taps outside the grid read zeros, so both enter unconditionally
        const float ex = PZ ? fmaf(hwx, hc.zb, fmaf(1.0f - hwx, hc.za, 0.0f)) : join(hI0, hwx, hc.za, hc.zb);
        pl[G.hslot] = hin ? omega * (hc.r * C.hinv) + ex : 0.0f;
      }
      if constexpr (PZ) {
        // the ring slot written here is not read in this iteration
        if (Pnext != Pcur) cstore(Pnext, pf);
        zplane(k + 2);
        const int Pn2 = ptopL(k + 4);
        if (Pn2 != Pnext) cload(Pn2, pf);
        Pcur = Pnext;
        Pnext = Pn2;
      }
      __syncthreads();
      float left, right;
      quad_xnb<float>(G, pl, uc, left, right);
      if (nv > 0) {
        float q[4], so[4];
        MG0_STENCIL_LDS(C, um, uc, un, pl, left, right, q)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          so[e] = fmaf(omega, (rc[e] - q[e]) * C.inv[e], uc[e]);
          if (!ML && in_quad<VEC>(e, nv)) acc = __fma_rn((double)rc[e], (double)so[e], acc);
        }
        // the finest level's s is next read by the A.p sweep, far beyond any cache: streamed;
        // a coarser level's correction is read soon by the finer level's interpolation
        if constexpr (ML) st4<float, VEC>(SO, (long long)(k - 1) * n2 + rowoff, nv, so);
        else st4_stream<float, VEC>(SO, (long long)(k - 1) * n2 + rowoff, nv, so);
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        um[e] = uc[e];
        uc[e] = un[e];
        rc[e] = qn.r[e];
      }
      qn = qnn;
      hc = hn;
      buf ^= 1;
    }
    if (!ML) {  // r^T s partial of the tile
      for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
      __syncthreads();
      if (threadIdx.x == 0) part[item].g[2] = red[0] + red[1] + red[2] + red[3];
    }
  }
}
#undef MG0_STENCIL
#undef MG0_STENCIL_LDS
#undef MG0_ITEM_SETUP

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct MgLevelHost {
  const Problem* prob = nullptr;
  Batch B;                 // the group's solves on this level's grid
  int n = 0;
  long long ndof = 0;
  DevBuf ci, cwd, cwf, lohi;  // transfer to the next level
  DevBuf vb, ve, ve2, vt;     // level vectors (levels >= 1), group-contiguous
  DevBuf vtx;                 // z/y-interpolated coarse correction (fine rows x coarse columns)
  DevBuf fine;                // MgFine of this level (levels >= 1 with a coarser level)
  bool quad = false;          // n % 4 == 0 and every vector offset a multiple of 4
  bool rows = false;          // the level's tiles span whole rows
  bool fz = false;            // its FP32 post-smoothing interpolates the coarse correction itself
  std::vector<int> ci_h;      // host copy of ci (transfer to the next level)
};

struct MgGroup {
  int q = 0, seg = 0;  // problem index; its segment in the V-cycle solve list
  std::vector<int> sol;
  DevBuf sid, off0;
  std::vector<MgLevelHost*> lv;    // this batch's levels, finest first (a prefix of lvpool)
  std::vector<MgLevelHost*> lvpool;  // owned; kept across batches so their buffers are reused
  DevBuf L;
  DevBuf Linv;  // FP32 V-cycle: the coarsest operator's inverse per solve (FP64)
  int mc = 0;
  ~MgGroup() {
    for (MgLevelHost* l : lvpool) delete l;
  }
};

struct MgRun {
  int nu = 1, device = 0;
  double omega = 6.0 / 7.0;
  bool fp32 = false;
  bool fused = false;  // level-0 correction + post-smoothing + r^T s in one tile kernel
  bool rx0 = false;    // FP32 fused: level-0 tiles span whole rows, the pre-smoothing forms the x-sums
  bool fz0 = false;    // FP32 fused: the level-0 post-smoothing interpolates the coarse correction itself
  std::vector<MgGroup*> g;     // one per problem of this batch (a prefix of gpool)
  std::vector<MgGroup*> gpool;  // owned; kept across batches so their buffers are reused
  DevBuf fine;    // MgFine per problem
  DevBuf x0, t0;  // level-0 scratch, laid out like the batch (x0 only without the fused kernels)
  ~MgRun() {
    for (MgGroup* q : gpool) delete q;
  }
};

// coarse problems, created once per (device, description, n) and kept
static const Problem* coarse_problem(const Problem* P, int n) {
  if (n == P->n) return P;
  struct Ent {
    int device, n, kind, f_kind;
    double gw;
    std::vector<int> blocks;
    Problem* prob;
  };
  static std::vector<Ent*> cache;
  for (Ent* e : cache)
    if (e->device == P->device && e->n == n && e->kind == P->desc.kind && e->f_kind == P->desc.f_kind &&
        e->gw == P->desc.gauss_width && e->blocks == P->blocks)
      return e->prob;
  rbws_problem_desc d = P->desc;
  d.n = n;
  d.blocks = P->blocks.empty() ? nullptr : P->blocks.data();
  Ent* e = new Ent{P->device, n, P->desc.kind, P->desc.f_kind, P->desc.gauss_width, P->blocks, nullptr};
  e->prob = problem_create(&d, P->device);
  cache.push_back(e);
  return e->prob;
}

static MgLv view(const MgLevelHost& l, const MgGroup& g, bool level0, bool fp32) {
  MgLv v;
  v.pd = (const ProbDev*)l.B.pd.ptr;
  v.sd = (const SolveDev*)l.B.sd.ptr;
  v.kap = fp32 ? l.B.kap32.ptr : l.B.kap64.ptr;
  v.voff = level0 ? (const long long*)g.off0.ptr : nullptr;
  v.sid = (const int*)g.sid.ptr;
  v.ndof = l.ndof;
  v.n = l.n;
  v.nsol = (int)g.sol.size();
  return v;
}

MgRun* mg_prepare(Batch& B, int nu, double omega, bool fp32, hipStream_t s) {
  // The hierarchy's objects and device buffers persist across batches (never
  // freed at exit): a later batch reuses every buffer that is large enough, so
  // repeated solves of a batch allocate nothing here.
  static thread_local MgRun* run = nullptr;
  if (run != nullptr && run->device != B.device) {
    delete run;
    run = nullptr;
  }
  if (run == nullptr) run = new MgRun();
  MgRun* m = run;
  m->g.clear();
  m->nu = nu;
  m->omega = omega;
  m->fp32 = fp32;
  m->device = B.device;
  const size_t el = fp32 ? sizeof(float) : sizeof(double);
  m->t0.get(el * std::max<long long>(B.total, 1), B.device);
  for (int q = 0; q < B.nprob; q++) {
    if ((int)m->gpool.size() <= q) m->gpool.push_back(new MgGroup());
    MgGroup* g = m->gpool[q];
    m->g.push_back(g);
    g->q = q;
    g->seg = 0;
    g->sol.clear();
    g->lv.clear();
    g->mc = 0;
    for (int b = 0; b < B.nsolve; b++) {
      if (B.sd_h[b].prob == q) g->sol.push_back(b);
      if (B.sd_h[b].prob < q) g->seg++;
    }
    if (g->sol.empty()) continue;
    const int ns = (int)g->sol.size();
    const Problem* P = B.probs[q];
    std::vector<long long> off(ns);
    std::vector<double> th((size_t)ns * P->Q);
    for (int t = 0; t < ns; t++) {
      off[t] = B.sd_h[g->sol[t]].off;
      for (int k = 0; k < P->Q; k++) th[(size_t)t * P->Q + k] = B.theta_h[(size_t)g->sol[t] * kMaxQ + k];
    }
    RBWS_HIP(hipMemcpyAsync(g->sid.get(sizeof(int) * ns, B.device), g->sol.data(), sizeof(int) * ns,
                            hipMemcpyHostToDevice, s));
    RBWS_HIP(hipMemcpyAsync(g->off0.get(sizeof(long long) * ns, B.device), off.data(), sizeof(long long) * ns,
                            hipMemcpyHostToDevice, s));
    int nl[16];
    const int L = mg_levels_of(P->n, nl);
    for (int l = 0; l < L; l++) {
      if ((int)g->lvpool.size() <= l) g->lvpool.push_back(new MgLevelHost());
      MgLevelHost* lv = g->lvpool[l];
      g->lv.push_back(lv);
      lv->prob = coarse_problem(P, nl[l]);
      lv->n = nl[l];
      lv->ndof = (long long)nl[l] * nl[l] * nl[l];
      std::vector<const Problem*> pl{lv->prob};
      batch_setup(lv->B, pl, nullptr, ns, nullptr, P->p, s, th.data(), l > 0);
      if (l > 0) {
        lv->vb.get(el * ns * lv->ndof, B.device);
        lv->ve.get(el * ns * lv->ndof, B.device);
        lv->ve2.get(el * ns * lv->ndof, B.device);
        lv->vt.get(el * ns * lv->ndof, B.device);
      }
      if (l + 1 < L) lv->vtx.get(el * ns * (size_t)nl[l] * nl[l] * nl[l + 1], B.device);
      lv->quad = nl[l] % 4 == 0;
      if (l == 0)
        for (long long o : off) lv->quad = lv->quad && o % 4 == 0;
    }
    // transfer tables level l -> l+1
    for (int l = 0; l + 1 < L; l++) {
      const int nf = nl[l], nc = nl[l + 1];
      // the z-marching transfers and the FP32 post-smoothing's tap window assume
      // that ci grows by at most one per fine point
      RBWS_REQUIRE(2 * (nc + 1) <= nf + 1, RBWS_EINVAL, "multigrid coarsening ratio above 1/2");
      std::vector<int> ci(nf);
      std::vector<double> cw(nf);
      std::vector<float> cwf(nf);
      for (int i = 1; i <= nf; i++) {
        const long long I = ((long long)i * (nc + 1)) / (nf + 1);
        ci[i - 1] = (int)I;
        cw[i - 1] = (double)((long long)i * (nc + 1) - I * (nf + 1)) / (double)(nf + 1);
        cwf[i - 1] = (float)cw[i - 1];
      }
      std::vector<int2> lh(nc + 2, make_int2(1, 0));
      for (int I = 1; I <= nc; I++) {
        int lo = nf + 1, hi = 0;
        for (int i = 1; i <= nf; i++)
          if (ci[i - 1] == I - 1 || ci[i - 1] == I) {
            lo = std::min(lo, i);
            hi = std::max(hi, i);
          }
        lh[I] = make_int2(lo, hi);
        RBWS_REQUIRE(hi - lo + 1 <= kSpan, RBWS_EINVAL, "multigrid transfer wider than expected");
      }
      // the restriction stages the fine span of 4 coarse rows and of 64 coarse columns
      for (int I = 1; I <= nc; I++) {
        RBWS_REQUIRE(lh[std::min(I + 3, nc)].y - lh[I].x + 1 <= kRsRows &&
                         lh[std::min(I + kRyJ - 1, nc)].y - lh[I].x + 1 <= kRyRows &&
                         lh[std::min(I + 63, nc)].y - lh[I].x + 1 <= kRsCols,
                     RBWS_EINVAL, "multigrid restriction block wider than expected");
      }
      MgLevelHost* lv = g->lv[l];
      lv->ci_h = ci;
      RBWS_HIP(hipMemcpyAsync(lv->ci.get(sizeof(int) * nf, B.device), ci.data(), sizeof(int) * nf,
                              hipMemcpyHostToDevice, s));
      RBWS_HIP(hipMemcpyAsync(lv->cwd.get(sizeof(double) * nf, B.device), cw.data(), sizeof(double) * nf,
                              hipMemcpyHostToDevice, s));
      RBWS_HIP(hipMemcpyAsync(lv->cwf.get(sizeof(float) * nf, B.device), cwf.data(), sizeof(float) * nf,
                              hipMemcpyHostToDevice, s));
      RBWS_HIP(hipMemcpyAsync(lv->lohi.get(sizeof(int2) * (nc + 2), B.device), lh.data(), sizeof(int2) * (nc + 2),
                              hipMemcpyHostToDevice, s));
      RBWS_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
    }
    // coarsest factors
    MgLevelHost* cl = g->lv[L - 1];
    g->mc = (int)cl->ndof;
    RBWS_REQUIRE(g->mc <= 27, RBWS_EINVAL, "coarsest multigrid level too large");
    double* Lf = (double*)g->L.get(sizeof(double) * (size_t)ns * g->mc * g->mc, B.device);
    RBWS_SCRATCH(badb);
    int* bad = (int*)badb.get(sizeof(int), B.device);
    RBWS_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    MgLv cv = view(*cl, *g, L == 1, false);  // (the factor kernel reads only tables)
    hipLaunchKernelGGL(k_mg_factor, dim3((ns + 63) / 64), dim3(64), 0, s, cv, Lf, bad);
    RBWS_HIP(hipGetLastError());
    int hb = 0;
    RBWS_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    RBWS_HIP(hipStreamSynchronize(s));
    RBWS_REQUIRE(hb == 0, RBWS_ENUMERIC, "coarsest multigrid operator not positive definite");
    if (fp32) {
      double* Li = (double*)g->Linv.get(sizeof(double) * (size_t)ns * g->mc * g->mc, B.device);
      const long long nth = (long long)ns * g->mc;
      hipLaunchKernelGGL(k_mg_inverse, dim3((unsigned)((nth + 63) / 64)), dim3(64), 0, s, cv, (const double*)Lf, Li);
      RBWS_HIP(hipGetLastError());
    }
  }
  // the fused level-0 post step needs nu = 1 and a coarse level for every problem
  m->fused = nu == 1;
  for (MgGroup* g : m->g)
    if (!g->sol.empty() && g->lv.size() < 2) m->fused = false;
  // tiles that span whole rows (at most 128 points, so n_c <= 63): the FP32
  // pre-smoothing forms the restriction's x-sums itself
  m->rx0 = fp32 && m->fused;
  for (int q = 0; q < B.nprob; q++) m->rx0 = m->rx0 && B.pd_h[q].ntx == 1 && B.probs[q]->n <= 128;
  for (MgGroup* g : m->g)
    for (MgLevelHost* lv : g->lv) lv->rows = lv->B.nsolve > 0 && lv->B.pd_h[0].ntx == 1 && lv->n <= 128;
  // ... and the FP32 post-smoothing interpolates the coarse correction itself
  // when its LDS rings hold what a tile needs
  auto pz_fits = [](const MgLevelHost& lv, int TY, int nc) {
    if (nc > 64) return false;
    const int CW = nc <= 16 ? 16 : nc <= 32 ? 32 : 64, n = lv.n;
    if ((TY + 2) * (CW + kPzPad) > kPzRows) return false;
    for (int j0 = 1; j0 <= n; j0 += TY) {
      const int Jb = lv.ci_h[std::max(j0 - 1, 1) - 1];
      if ((lv.ci_h[std::min(j0 + TY, n) - 1] + 2 - Jb) * CW > kPzRing) return false;
    }
    return true;
  };
  m->fz0 = m->rx0 && mg_pz_enabled();
  for (MgGroup* g : m->g) {
    for (MgLevelHost* lv : g->lv) lv->fz = false;
    if (g->sol.empty()) continue;
    for (size_t l = 1; fp32 && nu == 1 && mg_pz_enabled() && l + 1 < g->lv.size(); l++) {
      MgLevelHost& lv = *g->lv[l];
      lv.fz = lv.rows && pz_fits(lv, lv.B.pd_h[0].TY, g->lv[l + 1]->n);
    }
    if (g->lv.size() >= 2) m->fz0 = m->fz0 && pz_fits(*g->lv[0], B.pd_h[g->q].TY, g->lv[1]->n);
  }
  for (MgGroup* g : m->g)  // one launch covers every problem at level 0
    if (!g->sol.empty() && !g->lv.empty()) g->lv[0]->fz = m->fz0;
  std::vector<MgFine> fh(B.nprob);
  for (MgGroup* g : m->g) {
    if (g->sol.empty() || g->lv.size() < 2) continue;
    MgFine& f = fh[g->q];
    f.ezy = g->lv[0]->vtx.ptr;
    f.ci = (const int*)g->lv[0]->ci.ptr;
    f.cw = fp32 ? g->lv[0]->cwf.ptr : g->lv[0]->cwd.ptr;
    f.per = (long long)g->lv[0]->n * g->lv[0]->n * g->lv[1]->n;
    f.nc = g->lv[1]->n;
    f.fz = m->fz0 ? 1 : 0;
    f.lohi = (const int2*)g->lv[0]->lohi.ptr;
    f.ec = g->lv[1]->ve.ptr;
    // the same for the levels >= 1 that have a coarser level (FP32 fused path)
    for (size_t l = 1; fp32 && l + 1 < g->lv.size(); l++) {
      MgLevelHost& lv = *g->lv[l];
      MgFine fl{lv.vtx.ptr, (const int*)lv.ci.ptr, lv.cwf.ptr, (long long)lv.n * lv.n * g->lv[l + 1]->n,
                g->lv[l + 1]->n, lv.fz ? 1 : 0, (const int2*)lv.lohi.ptr, g->lv[l + 1]->ve.ptr};
      RBWS_HIP(hipMemcpy(lv.fine.get(sizeof(MgFine), B.device), &fl, sizeof(MgFine), hipMemcpyHostToDevice));
    }
  }
  RBWS_HIP(hipMemcpyAsync(m->fine.get(sizeof(MgFine) * fh.size(), B.device), fh.data(), sizeof(MgFine) * fh.size(),
                          hipMemcpyHostToDevice, s));
  if (!m->fused) m->x0.get(el * std::max<long long>(B.total, 1), B.device);
  RBWS_HIP(hipStreamSynchronize(s));
  return m;
}

static int g_mg_pz = 1;
bool mg_pz_enabled() { return g_mg_pz != 0; }
void set_mg_pz(int on) { g_mg_pz = on ? 1 : 0; }

static unsigned grid_for(long long items) {
  const long long g = std::min<long long>(std::max<long long>(items, 1), 65536);
  return (unsigned)((g + 7) & ~7LL);
}

// one V-cycle at level l of group g.  With `pre_only` (level 0 of the fused
// path, nu = 1) the residual after pre-smoothing is already in tres (written
// by k_mg_pre0, `scratch` unused) and the cycle stops once the z/y-interpolated
// coarse correction is in the level's vtx; k_mg_post0 finishes it.
template <typename T>
static void vcycle(MgRun* m, MgGroup& g, int l, const T* b, T* e, T* scratch, T* tres, MgList ml, hipStream_t s,
                   bool pre_only = false) {
  const bool pre_done = pre_only && l == 0;
  MgLevelHost& lv = *g.lv[l];
  const int ns = (int)g.sol.size();
  const bool l0 = l == 0;
  const MgLv v = view(lv, g, l0, m->fp32);
  if (l + 1 == (int)g.lv.size()) {
    if constexpr (sizeof(T) == 4) {
      if (m->fp32) {
        hipLaunchKernelGGL(k_mg_coarse_inv, dim3(ns), dim3(64), 0, s, v, ml, (const double*)g.Linv.ptr, b, e);
        return;
      }
    }
    hipLaunchKernelGGL(k_mg_coarse<T>, dim3(ns), dim3(64), 0, s, v, ml, (const double*)g.L.ptr, b, e);
    return;
  }
  const dim3 grid(grid_for((long long)ns * ((lv.ndof + 255) / 256)));
  const dim3 gq(grid_for((long long)ns * ((lv.ndof / 4 + 255) / 256)));
  const T om = (T)m->omega;
  // FP32, nu = 1, levels >= 1: fused tile kernels over every tile of the listed solves
  const bool tiles = m->fp32 && m->nu == 1 && l >= 1;
  // the pre-smoothing kernel forms the restriction's x-sums (whole-row tiles)
  const bool rx = l == 0 ? pre_only && m->rx0 : tiles && lv.rows;
  const int ntiles = lv.B.nsolve > 0 ? lv.B.sd_h[0].ntiles : 0;
  const int ktab = (lv.B.kap_max + 3) & ~3;
  const dim3 tgrid(8u * (unsigned)(((long long)ns * ntiles + 7) / 8));
  const size_t tlds = sizeof(float) * (ktab + 2 * QPLANE);
  auto smooth = [&](const T* ein, T* out) {
    if (lv.quad) hipLaunchKernelGGL((k_mg_quad<T, false>), gq, dim3(256), 0, s, v, ml, b, ein, out, om);
    else hipLaunchKernelGGL((k_mg_point<T, false>), grid, dim3(256), 0, s, v, ml, b, ein, out, om);
  };
  // 2 nu Jacobi writes alternate between `scratch` and `e`, the last one into e
  T* w[2] = {scratch, e};
  int wi = 0;
  if (tiles) {
    auto k = rx ? (lv.B.vec ? k_mg_pre0_32<true, true, true> : k_mg_pre0_32<false, true, true>)
                : (lv.B.vec ? k_mg_pre0_32<true, true, false> : k_mg_pre0_32<false, true, false>);
    hipLaunchKernelGGL(k, tgrid, dim3(256), tlds, s, (const int2*)lv.B.items.ptr, ml.list, ml.cnt, ntiles,
                       (const SolveDev*)lv.B.sd.ptr, (const ProbDev*)lv.B.pd.ptr, (const float*)lv.B.kap32.ptr,
                       (const float*)b, (float*)tres, (const MgFine*)lv.fine.ptr, nullptr, (float)m->omega, ktab);
  } else if (!pre_done) {
    smooth(nullptr, w[wi]);
    for (int it = 1; it < m->nu; it++) {
      smooth(w[wi], w[wi ^ 1]);
      wi ^= 1;
    }
    if (lv.quad) hipLaunchKernelGGL((k_mg_quad<T, true>), gq, dim3(256), 0, s, v, ml, b, (const T*)w[wi], tres, om);
    else hipLaunchKernelGGL((k_mg_point<T, true>), grid, dim3(256), 0, s, v, ml, b, (const T*)w[wi], tres, om);
  }
  MgLevelHost& cl = *g.lv[l + 1];
  const MgLv cv = view(cl, g, false, m->fp32);
  const T* cw = m->fp32 ? (const T*)lv.cwf.ptr : (const T*)lv.cwd.ptr;
  const T scale = (T)((double)(cl.n + 1) / (double)(lv.n + 1));
  const long long nrs = (long long)((cl.n + kRsSeg - 1) / kRsSeg) * ((cl.n + 3) / 4) * ((cl.n + 63) / 64);
  const long long nry = (long long)((cl.n + kRsSeg - 1) / kRsSeg) * ((cl.n + kRyJ - 1) / kRyJ) * ((cl.n + 63) / 64);
  const long long npyz = (long long)((lv.n + kPzSeg - 1) / kPzSeg) * ((lv.n + 3) / 4) * ((cl.n + 63) / 64);
  if (rx)
    hipLaunchKernelGGL(k_mg_restrict_yz<T>, dim3(grid_for((long long)ns * nry)), dim3(256), 0, s, v, cv, ml,
                       (const int*)lv.ci.ptr, cw, (const int2*)lv.lohi.ptr, (const T*)lv.vtx.ptr, (T*)cl.vb.ptr,
                       scale);
  else
    hipLaunchKernelGGL(k_mg_restrict<T>, dim3(grid_for((long long)ns * nrs)), dim3(256), 0, s, v, cv, ml,
                       (const int*)lv.ci.ptr, cw, (const int2*)lv.lohi.ptr, (const T*)tres, (T*)cl.vb.ptr, scale);
  vcycle<T>(m, g, l + 1, (const T*)cl.vb.ptr, (T*)cl.ve.ptr, (T*)cl.ve2.ptr, (T*)cl.vt.ptr, ml, s);
  // z/y interpolation of the coarse correction (into vtx, free again after the
  // restriction), unless the level's FP32 post-smoothing does it itself
  if (!lv.fz)
    hipLaunchKernelGGL(k_mg_pyz<T>, dim3(grid_for((long long)ns * npyz)), dim3(256), 0, s, v, cv, ml,
                       (const int*)lv.ci.ptr, cw, (const T*)cl.ve.ptr, (T*)lv.vtx.ptr);
  if (pre_only) return;
  if (tiles) {
    auto k = lv.fz ? (lv.B.vec ? k_mg_post0_32<true, true, true> : k_mg_post0_32<false, true, true>)
                   : (lv.B.vec ? k_mg_post0_32<true, true, false> : k_mg_post0_32<false, true, false>);
    hipLaunchKernelGGL(k, tgrid, dim3(256), tlds, s, (const int2*)lv.B.items.ptr, ml.list, ml.cnt, ntiles,
                       (const SolveDev*)lv.B.sd.ptr, (const ProbDev*)lv.B.pd.ptr, (const float*)lv.B.kap32.ptr,
                       (const MgFine*)lv.fine.ptr, nullptr, (const float*)b, (float*)e, nullptr, (float)m->omega,
                       ktab);
    return;
  }
  if (lv.quad)
    hipLaunchKernelGGL(k_mg_prolong_quad<T>, gq, dim3(256), 0, s, v, cv, ml, (const int*)lv.ci.ptr, cw,
                       (const T*)lv.vtx.ptr, w[wi]);
  else
    hipLaunchKernelGGL(k_mg_prolong<T>, grid, dim3(256), 0, s, v, cv, ml, (const int*)lv.ci.ptr, cw,
                       (const T*)lv.vtx.ptr, w[wi]);
  for (int it = 0; it < m->nu; it++) {
    smooth(w[wi], w[wi ^ 1]);
    wi ^= 1;
  }
  // 2 nu writes: the last one went to w[(2 nu - 1) & 1] = e
}

bool mg_apply(MgRun* m, Batch& B, const void* r, void* sv, const Lists& L, void* part, hipStream_t st) {
  const int ktab = (B.kap_max + 3) & ~3;
  const unsigned tgrid = 8u * (unsigned)((B.nitems + 7) / 8);
  KernelTimer& kt = ktimer();
  if (m->fused) {
    kt.begin(st, KK_MG_PRE);  // level 0: the residual after pre-smoothing into t0, over the tiles of the listed solves
    if (m->fp32) {
      auto k = m->rx0 ? (B.vec ? k_mg_pre0_32<true, false, true> : k_mg_pre0_32<false, false, true>)
                      : (B.vec ? k_mg_pre0_32<true, false, false> : k_mg_pre0_32<false, false, false>);
      hipLaunchKernelGGL(k, dim3(tgrid), dim3(256), sizeof(float) * (ktab + 2 * QPLANE), st, (const int2*)B.items.ptr,
                         (const int*)L.ap, (const int*)(L.cnt + WL_AP), 0, (const SolveDev*)B.sd.ptr,
                         (const ProbDev*)B.pd.ptr, (const float*)B.kap32.ptr, (const float*)r,
                         (float*)m->t0.ptr, (const MgFine*)m->fine.ptr, (const int*)L.gidx, (float)m->omega, ktab);
    } else {
      auto k = B.vec ? k_mg_pre0<double, true> : k_mg_pre0<double, false>;
      hipLaunchKernelGGL(k, dim3(tgrid), dim3(256), sizeof(double) * (ktab + 2 * QPLANE), st,
                         (const int2*)B.items.ptr, (const int*)L.ap, (const int*)(L.cnt + WL_AP),
                         (const SolveDev*)B.sd.ptr, (const ProbDev*)B.pd.ptr, (const double*)B.kap64.ptr,
                         (const double*)r, (double*)m->t0.ptr, m->omega, ktab);
    }
    kt.end(st);
  }
  kt.begin(st, KK_MG);
  for (MgGroup* g : m->g) {
    if (g->sol.empty()) continue;
    RBWS_REQUIRE(g->q < WL_MAXPROB, RBWS_EINVAL, "too many problems in one multigrid batch");
    const MgList ml{L.mg + g->seg, L.cnt + WL_MG + g->q};
    if (m->fp32)
      vcycle<float>(m, *g, 0, (const float*)r, (float*)sv, (float*)m->x0.ptr, (float*)m->t0.ptr, ml, st, m->fused);
    else
      vcycle<double>(m, *g, 0, (const double*)r, (double*)sv, (double*)m->x0.ptr, (double*)m->t0.ptr, ml, st,
                     m->fused);
  }
  kt.end(st);
  if (m->fused) {  // e1 formed again from r; the tiles of the listed solves are the CG work list L.ap
    kt.begin(st, KK_MG_POST);
    const unsigned grid = tgrid;
    if (m->fp32) {
      auto k = m->fz0 ? (B.vec ? k_mg_post0_32<true, false, true> : k_mg_post0_32<false, false, true>)
                      : (B.vec ? k_mg_post0_32<true, false, false> : k_mg_post0_32<false, false, false>);
      hipLaunchKernelGGL(k, dim3(grid), dim3(256), sizeof(float) * (ktab + 2 * QPLANE), st,
                         (const int2*)B.items.ptr, (const int*)L.ap, (const int*)(L.cnt + WL_AP), 0,
                         (const SolveDev*)B.sd.ptr, (const ProbDev*)B.pd.ptr, (const float*)B.kap32.ptr,
                         (const MgFine*)m->fine.ptr, (const int*)L.gidx, (const float*)r,
                         (float*)sv, (IrPart*)part, (float)m->omega, ktab);
    } else {
      auto k = B.vec ? k_mg_post0<double, true> : k_mg_post0<double, false>;
      hipLaunchKernelGGL(k, dim3(grid), dim3(256), sizeof(double) * (ktab + 2 * QPLANE), st,
                         (const int2*)B.items.ptr, (const int*)L.ap, (const int*)(L.cnt + WL_AP),
                         (const SolveDev*)B.sd.ptr, (const ProbDev*)B.pd.ptr, (const double*)B.kap64.ptr,
                         (const MgFine*)m->fine.ptr, (const int*)L.gidx, (const double*)r, (double*)sv, part,
                         m->omega, ktab);
    }
    kt.end(st);
  }
  RBWS_HIP(hipGetLastError());
  return m->fused;
}

void mg_apply_all(Batch& B, int nu, double omega, bool fp32, const void* r, void* sv, hipStream_t st) {
  if (B.nsolve == 0) return;
  RBWS_REQUIRE(B.nprob <= WL_MAXPROB, RBWS_EINVAL, "too many problems in one multigrid batch");
  Lists L = lists_init(B, st);
  // every tile on the ap list, every solve on its problem's V-cycle list
  const int ni = B.nitems, ns = B.nsolve;
  static thread_local std::vector<int> head, ap, mg;  // kept until the stream is synchronised below
  head.assign(64, 0);
  head[WL_AP] = ni;
  std::vector<int> seg(B.nprob + 1, 0);
  for (int b = 0; b < ns; b++) seg[B.sd_h[b].prob + 1]++;
  for (int q = 0; q < B.nprob; q++) {
    head[WL_MG + q] = seg[q + 1];
    seg[q + 1] += seg[q];
    head[WL_SEG + q] = seg[q];
  }
  ap.resize(ni);
  for (int t = 0; t < ni; t++) ap[t] = t;
  mg.resize(ns);
  for (int q = 0; q < B.nprob; q++)
    for (int i = 0; i < seg[q + 1] - seg[q]; i++) mg[seg[q] + i] = i;
  RBWS_HIP(hipMemcpyAsync(L.cnt, head.data(), sizeof(int) * head.size(), hipMemcpyHostToDevice, st));
  RBWS_HIP(hipMemcpyAsync(L.ap, ap.data(), sizeof(int) * ni, hipMemcpyHostToDevice, st));
  RBWS_HIP(hipMemcpyAsync(L.mg, mg.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
  MgRun* m = mg_prepare(B, nu, omega, fp32, st);
  RBWS_SCRATCH(part);
  void* pp = part.get(std::max(sizeof(CrAcc) * kSlots, sizeof(IrPart)) * (size_t)ni, B.device);
  mg_apply(m, B, r, sv, L, pp, st);
  RBWS_HIP(hipStreamSynchronize(st));
}

}  // namespace rbws
