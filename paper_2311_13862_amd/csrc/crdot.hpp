// crdot.hpp -- correctly rounded inner products on gfx950.
//
// Every inner product of the FP64 path is defined as the exact sum of the
// exact products, rounded once to nearest-even.  That makes the result
// independent of how the sum is split over lanes, waves and workgroups, so
// the GPU reproduces a sequential definition bit for bit.
//
// Fast path (every lane, every element):
//   p = x*y, e = fma(x,y,-p)        exact product p+e (TwoProd)
//   (s, es) = TwoSum(s, p)          exact running sum of the leading parts
//   lo += e + es                    the only rounded operations
//   ab += |e+es| + |lo|             bound: |exact - (s+lo)| <= 2^-53 * ab
// Partial accumulators combine the same way (combine()).  finalize() rounds
// s+lo and proves, from the bound, that no rounding boundary lies within the
// error interval; if it cannot (probability ~ n * 2^-53 per dot), the caller
// recomputes the dot exactly with the integer accumulator below.
//
// Exact path: a fixed-point accumulator of 32-bit digits held in 64-bit
// signed words (headroom for 2^31 additions per word), covering every
// product of two doubles (2^-2148 .. 2^2048).  Products are formed from the
// integer significands, so subnormals and underflowing products are exact.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbws {

struct CrAcc {
  double s, lo, ab;
};

__device__ __forceinline__ CrAcc cr_zero() { return CrAcc{0.0, 0.0, 0.0}; }

// products below this magnitude may have an inexact fma error term
#define RBWS_CR_TINY 0x1p-960

__device__ __forceinline__ void cr_add_prod(CrAcc& a, double x, double y) {
  double p = x * y;
  double e = __fma_rn(x, y, -p);
  double s = a.s + p;
  double bp = s - a.s;
  double es = (a.s - (s - bp)) + (p - bp);
  a.s = s;
  double t = e + es;
  double lo = a.lo + t;
  a.lo = lo;
  a.ab += fabs(t) + fabs(lo);
  if (fabs(p) < RBWS_CR_TINY && p != 0.0) a.ab = __builtin_inf();
}

__device__ __forceinline__ void cr_add(CrAcc& a, double p) {
  double s = a.s + p;
  double bp = s - a.s;
  double es = (a.s - (s - bp)) + (p - bp);
  a.s = s;
  double lo = a.lo + es;
  a.lo = lo;
  a.ab += fabs(es) + fabs(lo);
}

__device__ __forceinline__ CrAcc cr_combine(const CrAcc& a, const CrAcc& b) {
  double s = a.s + b.s;
  double bp = s - a.s;
  double es = (a.s - (s - bp)) + (b.s - bp);
  double t = a.lo + b.lo;
  double t2 = t + es;
  CrAcc r;
  r.s = s;
  r.lo = t2;
  r.ab = (a.ab + b.ab) + (fabs(t) + fabs(t2));
  return r;
}

__device__ __forceinline__ CrAcc cr_shfl_xor(const CrAcc& a, int m) {
  CrAcc r;
  r.s = __shfl_xor(a.s, m, 64);
  r.lo = __shfl_xor(a.lo, m, 64);
  r.ab = __shfl_xor(a.ab, m, 64);
  return r;
}

__device__ __forceinline__ CrAcc cr_wave_reduce(CrAcc a) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) a = cr_combine(a, cr_shfl_xor(a, m));
  return a;
}

// Reduce over the workgroup; the result is valid in thread 0.
// `sh` must hold blockDim.x/64 entries.
__device__ __forceinline__ CrAcc cr_block_reduce(CrAcc a, CrAcc* sh) {
  a = cr_wave_reduce(a);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    CrAcc r = sh[0];
    for (int i = 1; i < nw; i++) r = cr_combine(r, sh[i]);
    a = r;
  }
  return a;
}

__device__ __forceinline__ uint64_t dbits(double x) { return __double_as_longlong(x); }

// Distance from |h| to the next larger / smaller double (h finite, normal).
__device__ __forceinline__ double ulp_up(double a) {
  return __longlong_as_double(dbits(a) + 1) - a;
}
__device__ __forceinline__ double ulp_dn(double a) {
  return a - __longlong_as_double(dbits(a) - 1);
}

// Round the accumulated value.  Returns true and the correctly rounded value
// when the error bound proves it; false when the exact path is needed.
__device__ __forceinline__ bool cr_finalize(const CrAcc& a, double* out) {
  if (!(__builtin_isfinite(a.s) && __builtin_isfinite(a.lo) && __builtin_isfinite(a.ab)))
    return false;
  double hi = a.s + a.lo;
  double bp = hi - a.s;
  double lo = (a.s - (hi - bp)) + (a.lo - bp);  // s + lo_acc == hi + lo exactly
  double E = a.ab * 0x1p-53 * (1.0 + 0x1p-20);
  if (hi == 0.0) {
    if (lo == 0.0 && a.ab == 0.0) { *out = 0.0; return true; }
    return false;
  }
  double mag = fabs(hi);
  if (!(mag >= 0x1p-1000 && mag <= 0x1p+1000)) return false;
  double sl = hi > 0.0 ? lo : -lo;  // offset of the exact value away from 0
  double gu = ulp_up(mag), gd = ulp_dn(mag);
  const double k = 0.5 * (1.0 - 0x1p-40);
  if (sl + E < k * gu && sl - E > -k * gd) { *out = hi; return true; }
  return false;
}

// ----------------------------------------------------------------------------
// exact accumulator in LDS
// value = sum_i w[i] * 2^(32 i - XA_BIAS)
// ----------------------------------------------------------------------------
#define XA_WORDS 140
#define XA_BIAS 2240

struct XAcc {
  unsigned long long w[XA_WORDS];
  int bad;
};

__device__ __forceinline__ void xa_clear(XAcc* x) {
  for (int i = threadIdx.x; i < XA_WORDS; i += blockDim.x) x->w[i] = 0ull;
  if (threadIdx.x == 0) x->bad = 0;
}

// sig * 2^ex with sig < 2^53 (ex = -1074 for subnormals)
__device__ __forceinline__ void xa_decode(double v, uint64_t* sig, int* ex, bool* neg) {
  uint64_t b = dbits(v);
  *neg = (b >> 63) != 0;
  int be = (int)((b >> 52) & 0x7ff);
  uint64_t f = b & 0xfffffffffffffull;
  if (be == 0) { *sig = f; *ex = -1074; }
  else { *sig = f | 0x10000000000000ull; *ex = be - 1075; }
}

// add +/- (hi:lo) * 2^ex where hi:lo is a 128-bit magnitude
__device__ __forceinline__ void xa_add_mag(XAcc* x, uint64_t hi, uint64_t lo, int ex, bool neg) {
  int pos = ex + XA_BIAS;
  int word = pos >> 5, sh = pos & 31;
  uint32_t ch[4] = {(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
#pragma unroll
  for (int c = 0; c < 4; c++) {
    if (ch[c] == 0) continue;
    uint64_t v = (uint64_t)ch[c] << sh;  // < 2^63
    long long a0 = (long long)(v & 0xffffffffull), a1 = (long long)(v >> 32);
    if (neg) { a0 = -a0; a1 = -a1; }
    if (a0) atomicAdd(&x->w[word + c], (unsigned long long)a0);
    if (a1) atomicAdd(&x->w[word + c + 1], (unsigned long long)a1);
  }
}

__device__ __forceinline__ void xa_add(XAcc* x, double v) {
  if (!__builtin_isfinite(v)) { x->bad = 1; return; }
  if (v == 0.0) return;
  uint64_t s; int e; bool ng;
  xa_decode(v, &s, &e, &ng);
  xa_add_mag(x, 0ull, s, e, ng);
}

__device__ __forceinline__ void xa_add_prod(XAcc* x, double a, double b) {
  if (!__builtin_isfinite(a) || !__builtin_isfinite(b)) { x->bad = 1; return; }
  if (a == 0.0 || b == 0.0) return;
  uint64_t sa, sb; int ea, eb; bool na, nb;
  xa_decode(a, &sa, &ea, &na);
  xa_decode(b, &sb, &eb, &nb);
  uint64_t lo = sa * sb, hi = __umul64hi(sa, sb);
  xa_add_mag(x, hi, lo, ea + eb, na != nb);
}

// Round to nearest-even.  Single thread; the accumulator must be complete
// (call after a __syncthreads()).  Uses `dig` (XA_WORDS uint32 of scratch).
__device__ inline double xa_round(const XAcc* x, uint32_t* dig) {
  if (x->bad) return __builtin_nan("");
  long long carry = 0;
  for (int i = 0; i < XA_WORDS; i++) {
    long long t = (long long)x->w[i] + carry;
    dig[i] = (uint32_t)(t & 0xffffffffll);
    carry = (t - (long long)dig[i]) >> 32;  // exact floor division by 2^32
  }
  bool neg = carry < 0;
  if (neg) {  // |value| = 2^(32 W) - D
    uint64_t c = 1;
    for (int i = 0; i < XA_WORDS; i++) {
      uint64_t t = (uint64_t)(~dig[i]) + c;
      dig[i] = (uint32_t)t;
      c = t >> 32;
    }
  }
  int top = XA_WORDS - 1;
  while (top >= 0 && dig[top] == 0) top--;
  if (top < 0) return 0.0;
  int msb = top * 32 + (31 - __clz(dig[top]));
  int keep = msb - 52;                       // lowest kept bit (53 bits)
  if (keep < XA_BIAS - 1074) keep = XA_BIAS - 1074;
  // gather bits [keep, msb] and the round/sticky information
  uint64_t m = 0;
  for (int b = msb; b >= keep; b--) m = (m << 1) | ((dig[b >> 5] >> (b & 31)) & 1u);
  int rb = keep > 0 ? (int)((dig[(keep - 1) >> 5] >> ((keep - 1) & 31)) & 1u) : 0;
  bool st = false;
  int lb = keep - 2;
  if (lb >= 0) {
    int wd = lb >> 5;
    uint32_t mask = (lb & 31) == 31 ? 0xffffffffu : ((1u << ((lb & 31) + 1)) - 1u);
    if (dig[wd] & mask) st = true;
    for (int i = 0; i < wd && !st; i++) if (dig[i]) st = true;
  }
  if (rb && (st || (m & 1ull))) m++;
  double r = ldexp((double)m, keep - XA_BIAS);
  return neg ? -r : r;
}

}  // namespace rbws
