// mlp.hip -- the learned start on gfx950: a multilayer perceptron whose
// products run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, trained by backpropagation and Adam on FP32 master weights.
//
// Not part of the paper's method (its introduction cites neural-network
// initial guesses as related work); it predicts the reduced coefficients c(mu)
// that the Galerkin solve would produce, so the lift V c gives a start without
// the reduced solve.  The reduced solve stays as the fallback.
//
// Layouts (every size padded to a multiple of 32 with zeros, so that the MFMA
// operands are whole 16-byte rows and padding contributes nothing):
//   activations H_l: rows = batch, K-contiguous (the A operand of the next
//   layer); W_l: out x in, K-contiguous (the B operand, C = A B^T).  For the
//   weight gradients dW_l = G_l^T H_{l-1} the batch is the reduction axis, so
//   the forward pass also writes H_l^T and the loss/backward steps G^T; the
//   input gradient dH = G_l W_l reads a transposed BF16 copy W_l^T that the
//   optimiser refreshes with W_l.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "mlp.hpp"

namespace rbws {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static inline int pad32(int v) { return (v + 31) & ~31; }

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct InScale {
  int p, log_cols;
  double in_m, in_s, lin_c, lin_hw, out_pow;
};

__device__ __forceinline__ double log_mean(const double* mu, const InScale& S) {
  double l = 0.0;
  for (int i = 0; i < S.log_cols; i++) l += log10(mu[i]);
  return S.log_cols > 0 ? l / S.log_cols : 0.0;
}

// X[r][i] (bf16, rows x ld) from mu (nrow x p); zero padding
__global__ void k_mlp_in(const double* __restrict__ mu, int nrow, int rows, int ld, InScale S,
                         __bf16* __restrict__ X) {
  const long long tot = (long long)rows * ld;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / ld), i = (int)(e % ld);
    float v = 0.0f;
    if (r < nrow && i < S.p) {
      const double m = mu[(long long)r * S.p + i];
      v = (float)(i < S.log_cols ? (log10(m) - S.in_m) / S.in_s : (m - S.lin_c) / S.lin_hw);
    }
    X[e] = (__bf16)v;
  }
}

// scaled targets Y[r][j] = (c 10^(out_pow l(mu)) - mean_j) / std_j (float, zero padding)
__global__ void k_mlp_tgt(const double* __restrict__ mu, const double* __restrict__ c, int nrow, int nout,
                          int ld, InScale S, const double* __restrict__ scal, float* __restrict__ Y) {
  const long long tot = (long long)nrow * ld;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / ld), j = (int)(e % ld);
    float v = 0.0f;
    if (j < nout) {
      const double f = S.out_pow != 0.0 ? pow(10.0, S.out_pow * log_mean(mu + (long long)r * S.p, S)) : 1.0;
      v = (float)((c[(long long)r * nout + j] * f - scal[j]) / scal[nout + j]);
    }
    Y[e] = v;
  }
}

// mean and standard deviation of the scaled targets, one thread per output
__global__ void k_mlp_stats(const double* __restrict__ mu, const double* __restrict__ c, int nrow, int nout,
                            InScale S, double* __restrict__ scal) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nout) return;
  double s = 0.0;
  for (int r = 0; r < nrow; r++) {
    const double f = S.out_pow != 0.0 ? pow(10.0, S.out_pow * log_mean(mu + (long long)r * S.p, S)) : 1.0;
    s += c[(long long)r * nout + j] * f;
  }
  const double mean = s / nrow;
  double q = 0.0;
  for (int r = 0; r < nrow; r++) {
    const double f = S.out_pow != 0.0 ? pow(10.0, S.out_pow * log_mean(mu + (long long)r * S.p, S)) : 1.0;
    const double dv = c[(long long)r * nout + j] * f - mean;
    q += dv * dv;
  }
  const double sd = sqrt(q / nrow);
  scal[j] = mean;
  scal[nout + j] = sd > 0.0 ? sd : 1.0;
}

// c[rows[r]][j] = (mean_j + std_j y[r][j]) * 10^(-out_pow l(mu_r)) (double)
__global__ void k_mlp_outc(const float* __restrict__ y, int nrow, int ldy, int nout, const int* __restrict__ rows,
                           const double* __restrict__ mu, InScale S, const double* __restrict__ scal,
                           double* __restrict__ c, int cstride) {
  const long long tot = (long long)nrow * nout;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / nout), j = (int)(e % nout);
    const double f = S.out_pow != 0.0 ? pow(10.0, -S.out_pow * log_mean(mu + (long long)r * S.p, S)) : 1.0;
    const int dst = rows ? rows[r] : r;
    c[(long long)dst * cstride + j] = (scal[j] + scal[nout + j] * (double)y[(long long)r * ldy + j]) * f;
  }
}

// minibatch gather for step t: rows perm[e npairs + s nb + r], e = (t - t0) / spe, s = (t - t0) % spe
__global__ void k_mlp_gather(const AdamDev* __restrict__ ad, int t0, const int* __restrict__ perm, int npairs,
                             int nb, int cap, const __bf16* __restrict__ Xa, int ldx, const float* __restrict__ Ya,
                             int ldy, __bf16* __restrict__ X, __bf16* __restrict__ Xt, float* __restrict__ Y) {
  const int r = blockIdx.x;
  const int rel = ad->t - t0;
  const int src = r < nb ? perm[(long long)(rel / ad->spe) * npairs + (long long)(rel % ad->spe) * nb + r] : -1;
  for (int i = threadIdx.x; i < ldx; i += blockDim.x) {
    const __bf16 v = src >= 0 ? Xa[(long long)src * ldx + i] : (__bf16)0.0f;
    X[(long long)r * ldx + i] = v;
    Xt[(long long)i * cap + r] = v;
  }
  for (int j = threadIdx.x; j < ldy; j += blockDim.x) Y[(long long)r * ldy + j] = src >= 0 ? Ya[(long long)src * ldy + j] : 0.0f;
}

// ---------------------------------------------------------------------------
// C[M x N] = A[M x K] B[N x K]^T on the matrix cores, with fused epilogues.
// A workgroup of 4 waves computes a 32 x 32 tile, one 16 x 16 block per wave;
// lane l feeds row l % 16 and the 8 K-values 8 (l / 16) .. +7 of both operands
// and holds the outputs (4 (l / 16) + i, l % 16), i < 4.  M, N, K are
// multiples of 32 (padded); rows and columns are 16-byte aligned.
// ---------------------------------------------------------------------------
enum { EPI_HID = 0, EPI_OUT = 1, EPI_DH = 2, EPI_DW = 3 };
struct Epi {
  const float* bias;  // HID, OUT
  float* z;           // HID: pre-activations out (nullable); DH: pre-activations in
  __bf16* h;          // HID: H out; DH: G out (bf16)
  __bf16* ht;         // HID: H^T out (nullable); DH: G^T out
  float* o;           // OUT: y; DH: G (FP32); DW: dW
  int ld;             // leading dimension of z, h, o (= N)
  int ldt;            // leading dimension of ht (rows of the batch, padded)
  int mreal;          // HID, DH: rows >= mreal are written as zero
  int pad;
};

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                              const __bf16* __restrict__ Bm, int ldb, Epi e) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + (w >> 1) * 16, n0 = blockIdx.x * 32 + (w & 1) * 16;
  if (m0 >= M || n0 >= N) return;
  const int r = lane & 15, q = lane >> 4;
  const __bf16* pa = A + (long long)(m0 + r) * lda + 8 * q;
  const __bf16* pb = Bm + (long long)(n0 + r) * ldb + 8 * q;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k = 0; k < K; k += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(pa + k);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(pb + k);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  const int n = n0 + r;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int m = m0 + 4 * q + i;
    const long long at = (long long)m * e.ld + n;
    if (EPI == EPI_HID) {
      const float z = acc[i] + e.bias[n];
      const float h = m < e.mreal ? gelu_f(z) : 0.0f;
      if (e.z) e.z[at] = z;
      e.h[at] = (__bf16)h;
      if (e.ht) e.ht[(long long)n * e.ldt + m] = (__bf16)h;
    } else if (EPI == EPI_OUT) {
      e.o[at] = acc[i] + e.bias[n];
    } else if (EPI == EPI_DH) {
      const float gv = m < e.mreal ? acc[i] * gelu_grad_f(e.z[at]) : 0.0f;
      e.o[at] = gv;
      e.h[at] = (__bf16)gv;
      e.ht[(long long)n * e.ldt + m] = (__bf16)gv;
    } else {
      e.o[at] = acc[i];
    }
  }
}

// loss and the output gradient G = 2 (y - t) / (nb nout) (single workgroup)
__global__ __launch_bounds__(256) void k_mlp_mse(const float* __restrict__ y, const float* __restrict__ tg, int nb,
                                                 int nout, int ld, int cap, const AdamDev* __restrict__ ad, int t0,
                                                 int hist, float* __restrict__ g32, __bf16* __restrict__ gb,
                                                 __bf16* __restrict__ gt, double* __restrict__ loss) {
  __shared__ double red[256];
  const float sc = 2.0f / (float)((long long)nb * nout);
  double s = 0.0;
  const long long tot = (long long)cap * ld;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e / ld), j = (int)(e % ld);
    float gv = 0.0f;
    if (r < nb && j < nout) {
      const float dv = y[e] - tg[e];
      s += (double)dv * (double)dv;
      gv = sc * dv;
    }
    g32[e] = gv;
    gb[e] = (__bf16)gv;
    gt[(long long)j * cap + r] = (__bf16)gv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k >= 1; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[hist ? ad->t - t0 : 0] = red[0] / (double)((long long)nb * nout);
}

// db[n] = sum over the batch of G[r][n]
__global__ void k_mlp_colsum(const float* __restrict__ g32, int rows, int ld, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ld) return;
  double s = 0.0;
  for (int r = 0; r < rows; r++) s += (double)g32[(long long)r * ld + n];
  db[n] = (float)s;
}

// Adam on one layer (update != 0), then refresh the BF16 copies W and W^T;
// padding entries stay zero
struct LayerDev {
  long long wo, bo, wbo, wto;
  int out, in, outp, inp;
};
__global__ void k_mlp_adam(const AdamDev* __restrict__ ad, int t0, int update, LayerDev Ld, float* __restrict__ w,
                           float* __restrict__ mm, float* __restrict__ vv, const float* __restrict__ g,
                           __bf16* __restrict__ wb, __bf16* __restrict__ wt) {
  const long long nw = (long long)Ld.outp * Ld.inp, tot = nw + Ld.outp;
  float lr = 0.0f, c1 = 1.0f, c2 = 1.0f, b1 = 0.0f, b2 = 0.0f, eps = 0.0f;
  if (update) {
    const int rel = ad->t - t0;
    double l = ad->lr0;
    if (ad->T > 0) l = ad->lr_min + 0.5 * (ad->lr0 - ad->lr_min) * (1.0 + cos(3.14159265358979323846 * rel / ad->T));
    lr = (float)l;
    const int tt = ad->t + 1;
    c1 = (float)(1.0 - pow(ad->b1, tt));
    c2 = (float)(1.0 - pow(ad->b2, tt));
    b1 = (float)ad->b1;
    b2 = (float)ad->b2;
    eps = (float)ad->eps;
  }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    int o, i;
    long long at;
    if (e < nw) {
      o = (int)(e / Ld.inp);
      i = (int)(e % Ld.inp);
      at = Ld.wo + e;
    } else {
      o = (int)(e - nw);
      i = 0;
      at = Ld.bo + o;
    }
    const bool real = o < Ld.out && i < Ld.in;
    float wv = w[at];
    if (update && real) {
      const float gv = g[at];
      const float mv = b1 * mm[at] + (1.0f - b1) * gv;
      const float vv2 = b2 * vv[at] + (1.0f - b2) * gv * gv;
      mm[at] = mv;
      vv[at] = vv2;
      wv -= lr * (mv / c1) / (sqrtf(vv2 / c2) + eps);
      w[at] = wv;
    }
    if (e < nw) {
      const __bf16 hb = (__bf16)(real ? wv : 0.0f);
      wb[Ld.wbo + e] = hb;
      wt[Ld.wto + (long long)i * Ld.outp + o] = hb;
    }
  }
}

__global__ void k_mlp_tick(AdamDev* ad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ad->t += 1;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static InScale in_scale(const Mlp* m) {
  InScale S;
  S.p = m->d.p;
  S.log_cols = m->d.log_cols;
  S.in_m = m->d.in_m;
  S.in_s = m->d.in_s;
  S.lin_c = 0.5 * (m->d.lin_lo + m->d.lin_hi);
  S.lin_hw = 0.5 * (m->d.lin_hi - m->d.lin_lo);
  S.out_pow = m->d.out_pow;
  return S;
}

static LayerDev layer_dev(const Mlp* m, int l) {
  return LayerDev{m->wo[l], m->bo[l], m->wbo[l], m->wto[l], m->out[l], m->in[l], m->outp[l], m->inp[l]};
}

static unsigned blocks_for(long long n) { return (unsigned)std::min<long long>(std::max<long long>((n + 255) / 256, 1), 4096); }

static void ensure_ws(Mlp* m, int rows) {
  const int cap = pad32(std::max(rows, 32));
  if (cap <= m->cap) return;
  const int dev = m->device;
  const int L = m->L, W = m->maxw, K0 = m->inp[0], NO = m->outp[L - 1];
  m->cap = cap;
  m->x.get(sizeof(__bf16) * cap * K0, dev);
  m->xt.get(sizeof(__bf16) * cap * K0, dev);
  m->c.get(sizeof(float) * cap * NO, dev);
  m->o.get(sizeof(float) * cap * NO, dev);
  const long long hid = (long long)std::max(L - 1, 1) * cap * W;
  m->zs.get(sizeof(float) * hid, dev);
  m->hs.get(sizeof(__bf16) * hid, dev);
  m->hts.get(sizeof(__bf16) * hid, dev);
  m->g32.get(sizeof(float) * 2LL * cap * W, dev);
  m->gb.get(sizeof(__bf16) * 2LL * cap * W, dev);
  m->gt.get(sizeof(__bf16) * 2LL * cap * W, dev);
}

// forward over `cap` rows of m->x (the first `mreal` real); train: keep Z and H^T
static void forward(Mlp* m, int mreal, bool train, hipStream_t s) {
  const int cap = m->cap, L = m->L;
  const __bf16* A = (const __bf16*)m->x.ptr;
  int lda = m->inp[0];
  const __bf16* wb = (const __bf16*)m->wb.ptr;
  const float* w = (const float*)m->w.ptr;
  for (int l = 0; l < L; l++) {
    const int N = m->outp[l], K = m->inp[l];
    Epi e{};
    e.bias = w + m->bo[l];
    e.ld = N;
    e.ldt = cap;
    e.mreal = mreal;
    dim3 grid(N / 32, cap / 32);
    if (l < L - 1) {
      const long long off = (long long)l * cap * m->maxw;
      e.z = train ? (float*)m->zs.ptr + off : nullptr;
      e.h = (__bf16*)m->hs.ptr + off;
      e.ht = train ? (__bf16*)m->hts.ptr + off : nullptr;
      hipLaunchKernelGGL(k_gemm<EPI_HID>, grid, dim3(256), 0, s, cap, N, K, A, lda, wb + m->wbo[l], K, e);
      A = e.h;
      lda = N;
    } else {
      e.o = (float*)m->o.ptr;
      hipLaunchKernelGGL(k_gemm<EPI_OUT>, grid, dim3(256), 0, s, cap, N, K, A, lda, wb + m->wbo[l], K, e);
    }
  }
  RBWS_HIP(hipGetLastError());
}

// loss (into loss[slot]) and gradients of all parameters into m->g
static void backward(Mlp* m, int nb, const AdamDev* ad, int t0, int hist, double* loss, hipStream_t s) {
  const int cap = m->cap, L = m->L, W = m->maxw;
  float* g = (float*)m->g.ptr;
  float* g32 = (float*)m->g32.ptr;
  __bf16* gb = (__bf16*)m->gb.ptr;
  __bf16* gt = (__bf16*)m->gt.ptr;
  const long long half = (long long)cap * W;
  int cur = 0;
  hipLaunchKernelGGL(k_mlp_mse, dim3(1), dim3(256), 0, s, (const float*)m->o.ptr, (const float*)m->c.ptr, nb,
                     m->out[L - 1], m->outp[L - 1], cap, ad, t0, hist, g32, gb, gt, loss);
  for (int l = L - 1; l >= 0; l--) {
    const int NO = m->outp[l], NI = m->inp[l];
    const __bf16* Hprev_t = l > 0 ? (const __bf16*)m->hts.ptr + (long long)(l - 1) * cap * W
                                  : (const __bf16*)m->xt.ptr;
    Epi e{};
    e.o = g + m->wo[l];
    e.ld = NI;
    hipLaunchKernelGGL(k_gemm<EPI_DW>, dim3(NI / 32, NO / 32), dim3(256), 0, s, NO, NI, cap,
                       (const __bf16*)(gt + cur * half), cap, Hprev_t, cap, e);
    hipLaunchKernelGGL(k_mlp_colsum, dim3((NO + 255) / 256), dim3(256), 0, s, (const float*)(g32 + cur * half),
                       cap, NO, g + m->bo[l]);
    if (l > 0) {
      const int nxt = 1 - cur;
      Epi d{};
      d.z = (float*)m->zs.ptr + (long long)(l - 1) * cap * W;
      d.o = g32 + nxt * half;
      d.h = gb + nxt * half;
      d.ht = gt + nxt * half;
      d.ld = NI;
      d.ldt = cap;
      d.mreal = nb;
      hipLaunchKernelGGL(k_gemm<EPI_DH>, dim3(NI / 32, cap / 32), dim3(256), 0, s, cap, NI, NO,
                         (const __bf16*)(gb + cur * half), NO, (const __bf16*)m->wt.ptr + m->wto[l], NO, d);
      cur = nxt;
    }
  }
  RBWS_HIP(hipGetLastError());
}

static void adam_all(Mlp* m, int t0, int update, hipStream_t s) {
  for (int l = 0; l < m->L; l++) {
    const LayerDev Ld = layer_dev(m, l);
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for((long long)Ld.outp * Ld.inp + Ld.outp)), dim3(256), 0, s,
                       (const AdamDev*)m->ad.ptr, t0, update, Ld, (float*)m->w.ptr, (float*)m->m.ptr,
                       (float*)m->v.ptr, (const float*)m->g.ptr, (__bf16*)m->wb.ptr, (__bf16*)m->wt.ptr);
  }
  RBWS_HIP(hipGetLastError());
}

static AdamDev adam_host(const Mlp* m) {
  AdamDev a;
  RBWS_HIP(hipMemcpy(&a, m->ad.ptr, sizeof a, hipMemcpyDeviceToHost));
  return a;
}

static void zero_dev(DevBuf& b, size_t bytes, int dev, hipStream_t s) {
  std::vector<char> z(bytes, 0);
  RBWS_HIP(hipMemcpyAsync(b.get(bytes, dev), z.data(), bytes, hipMemcpyHostToDevice, s));
  RBWS_HIP(hipStreamSynchronize(s));
}

static void pack_to_padded(const Mlp* m, const float* params, std::vector<float>& pad) {
  pad.assign(m->npad, 0.0f);
  long long k = 0;
  for (int l = 0; l < m->L; l++) {
    for (int o = 0; o < m->out[l]; o++)
      for (int i = 0; i < m->in[l]; i++) pad[m->wo[l] + (long long)o * m->inp[l] + i] = params[k++];
    for (int o = 0; o < m->out[l]; o++) pad[m->bo[l] + o] = params[k++];
  }
}

static void padded_to_pack(const Mlp* m, const std::vector<float>& pad, float* params) {
  long long k = 0;
  for (int l = 0; l < m->L; l++) {
    for (int o = 0; o < m->out[l]; o++)
      for (int i = 0; i < m->in[l]; i++) params[k++] = pad[m->wo[l] + (long long)o * m->inp[l] + i];
    for (int o = 0; o < m->out[l]; o++) params[k++] = pad[m->bo[l] + o];
  }
}

static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

Mlp* mlp_create(const rbws_mlp_desc* d, int device, const float* params, unsigned long long seed) {
  RBWS_REQUIRE(d != nullptr, RBWS_EINVAL, "desc is NULL");
  RBWS_REQUIRE(d->p >= 1 && d->p <= 64, RBWS_EINVAL, "p must be in 1..64");
  RBWS_REQUIRE(d->nout >= 1 && d->nout <= 64, RBWS_EINVAL, "nout must be in 1..64");
  RBWS_REQUIRE(d->hidden >= 32 && d->hidden <= 1024 && d->hidden % 32 == 0, RBWS_EINVAL,
               "hidden must be a multiple of 32 in 32..1024");
  RBWS_REQUIRE(d->depth >= 1 && d->depth <= 8, RBWS_EINVAL, "depth must be in 1..8");
  RBWS_REQUIRE(d->log_cols >= 0 && d->log_cols <= d->p, RBWS_EINVAL, "log_cols must be in 0..p");
  RBWS_REQUIRE(d->in_s != 0.0 && std::isfinite(d->in_s) && std::isfinite(d->in_m), RBWS_EINVAL, "bad in_m/in_s");
  RBWS_REQUIRE(d->log_cols == d->p || d->lin_hi > d->lin_lo, RBWS_EINVAL, "lin_hi must exceed lin_lo");
  RBWS_REQUIRE(std::isfinite(d->out_pow), RBWS_EINVAL, "bad out_pow");
  RBWS_HIP(hipSetDevice(device));
  Mlp* m = new Mlp();
  try {
    m->device = device;
    m->d = *d;
    m->L = d->depth + 1;
    long long off = 0, offb = 0;
    for (int l = 0; l < m->L; l++) {
      const int in = l == 0 ? d->p : d->hidden, out = l == m->L - 1 ? d->nout : d->hidden;
      m->in.push_back(in);
      m->out.push_back(out);
      m->inp.push_back(pad32(in));
      m->outp.push_back(pad32(out));
      m->wo.push_back(off);
      off += (long long)pad32(out) * pad32(in);
      m->bo.push_back(off);
      off += pad32(out);
      m->wbo.push_back(offb);
      m->wto.push_back(offb);
      offb += (long long)pad32(out) * pad32(in);
      m->np += (long long)out * in + out;
      m->maxw = std::max({m->maxw, pad32(out), pad32(in)});
    }
    m->npad = off;
    m->nbf = offb;
    m->out_mean.assign(d->nout, 0.0);
    m->out_std.assign(d->nout, 1.0);
    hipStream_t s = nullptr;
    zero_dev(m->m, sizeof(float) * m->npad, device, s);
    zero_dev(m->v, sizeof(float) * m->npad, device, s);
    zero_dev(m->g, sizeof(float) * m->npad, device, s);
    m->wb.get(sizeof(__bf16) * m->nbf, device);
    m->wt.get(sizeof(__bf16) * m->nbf, device);
    AdamDev a{};
    a.spe = 1;
    a.lr0 = 1e-3;
    a.b1 = 0.9;
    a.b2 = 0.999;
    a.eps = 1e-8;
    RBWS_HIP(hipMemcpy(m->ad.get(sizeof(AdamDev), device), &a, sizeof a, hipMemcpyHostToDevice));
    mlp_set_scaling(m, nullptr, nullptr, s);
    std::vector<float> init;
    if (!params) {
      init.resize(m->np);
      uint64_t st = seed;
      long long k = 0;
      for (int l = 0; l < m->L; l++) {
        const double bound = 1.0 / std::sqrt((double)m->in[l]);
        for (long long e = 0; e < (long long)m->out[l] * m->in[l]; e++) {
          const double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;
          init[k++] = (float)((2.0 * u - 1.0) * bound);
        }
        for (int o = 0; o < m->out[l]; o++) init[k++] = 0.0f;
      }
      params = init.data();
    }
    mlp_set_params(m, params, s);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

void mlp_destroy(Mlp* m) {
  if (!m) return;
  if (m->own) (void)hipStreamDestroy(m->own);
  delete m;
}

void mlp_set_params(Mlp* m, const float* params, hipStream_t s) {
  RBWS_REQUIRE(params != nullptr, RBWS_EINVAL, "params is NULL");
  RBWS_HIP(hipSetDevice(m->device));
  std::vector<float> pad;
  pack_to_padded(m, params, pad);
  for (long long i = 0; i < m->np; i++) RBWS_REQUIRE(std::isfinite(params[i]), RBWS_EINVAL, "params must be finite");
  RBWS_HIP(hipMemcpyAsync(m->w.get(sizeof(float) * m->npad, m->device), pad.data(), sizeof(float) * m->npad,
                          hipMemcpyHostToDevice, s));
  std::vector<float> z(m->npad, 0.0f);
  RBWS_HIP(hipMemcpyAsync(m->m.ptr, z.data(), sizeof(float) * m->npad, hipMemcpyHostToDevice, s));
  RBWS_HIP(hipMemcpyAsync(m->v.ptr, z.data(), sizeof(float) * m->npad, hipMemcpyHostToDevice, s));
  AdamDev a;
  RBWS_HIP(hipMemcpyAsync(&a, m->ad.ptr, sizeof a, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  a.t = 0;
  RBWS_HIP(hipMemcpyAsync(m->ad.ptr, &a, sizeof a, hipMemcpyHostToDevice, s));
  adam_all(m, 0, 0, s);  // BF16 copies
  RBWS_HIP(hipStreamSynchronize(s));
}

void mlp_get_params(const Mlp* m, float* params, hipStream_t s) {
  RBWS_REQUIRE(params != nullptr, RBWS_EINVAL, "params is NULL");
  std::vector<float> pad(m->npad);
  RBWS_HIP(hipMemcpyAsync(pad.data(), m->w.ptr, sizeof(float) * m->npad, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  padded_to_pack(m, pad, params);
}

void mlp_set_scaling(Mlp* m, const double* mean, const double* stdev, hipStream_t s) {
  const int no = m->d.nout;
  for (int j = 0; j < no; j++) {
    const double a = mean ? mean[j] : 0.0, b = stdev ? stdev[j] : 1.0;
    RBWS_REQUIRE(std::isfinite(a) && std::isfinite(b) && b != 0.0, RBWS_EINVAL, "bad output scaling");
    m->out_mean[j] = a;
    m->out_std[j] = b;
  }
  std::vector<double> h(2 * no);
  for (int j = 0; j < no; j++) {
    h[j] = m->out_mean[j];
    h[no + j] = m->out_std[j];
  }
  RBWS_HIP(hipMemcpyAsync(m->scal.get(sizeof(double) * 2 * no, m->device), h.data(), sizeof(double) * 2 * no,
                          hipMemcpyHostToDevice, s));
  RBWS_HIP(hipStreamSynchronize(s));
}

static void check_mu(const Mlp* m, const double* mu, int n) {
  RBWS_REQUIRE(mu != nullptr, RBWS_EINVAL, "mu is NULL");
  for (long long r = 0; r < n; r++)
    for (int i = 0; i < m->d.p; i++) {
      const double v = mu[r * m->d.p + i];
      RBWS_REQUIRE(std::isfinite(v), RBWS_EINVAL, "mu must be finite");
      RBWS_REQUIRE(i >= m->d.log_cols || v > 0.0, RBWS_EINVAL, "log-scaled parameters must be positive");
    }
}

static double* upload_d(DevBuf& b, const double* h, long long n, int dev, hipStream_t s) {
  double* p = (double*)b.get(sizeof(double) * std::max<long long>(n, 1), dev);
  RBWS_HIP(hipMemcpyAsync(p, h, sizeof(double) * n, hipMemcpyHostToDevice, s));
  return p;
}

void mlp_fit_scaling(Mlp* m, const double* mu, const double* c, int npairs, hipStream_t s) {
  RBWS_REQUIRE(npairs >= 1 && c != nullptr, RBWS_EINVAL, "need pairs");
  check_mu(m, mu, npairs);
  RBWS_HIP(hipSetDevice(m->device));
  RBWS_SCRATCH(mub);
  RBWS_SCRATCH(cb);
  const double* md = upload_d(mub, mu, (long long)npairs * m->d.p, m->device, s);
  const double* cd = upload_d(cb, c, (long long)npairs * m->d.nout, m->device, s);
  hipLaunchKernelGGL(k_mlp_stats, dim3((m->d.nout + 63) / 64), dim3(64), 0, s, md, cd, npairs, m->d.nout,
                     in_scale(m), (double*)m->scal.ptr);
  RBWS_HIP(hipGetLastError());
  std::vector<double> h(2 * m->d.nout);
  RBWS_HIP(hipMemcpyAsync(h.data(), m->scal.ptr, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < m->d.nout; j++) {
    m->out_mean[j] = h[j];
    m->out_std[j] = h[m->d.nout + j];
  }
}

// inputs of `n` rows into m->x (the workspace holds at least n rows)
static void load_inputs(Mlp* m, const double* mu, int n, hipStream_t s, const double** mu_dev) {
  check_mu(m, mu, n);
  ensure_ws(m, n);
  RBWS_SCRATCH(mub);
  const double* md = upload_d(mub, mu, (long long)n * m->d.p, m->device, s);
  hipLaunchKernelGGL(k_mlp_in, dim3(blocks_for((long long)m->cap * m->inp[0])), dim3(256), 0, s, md, n, m->cap,
                     m->inp[0], in_scale(m), (__bf16*)m->x.ptr);
  RBWS_HIP(hipGetLastError());
  if (mu_dev) *mu_dev = md;
}

const float* mlp_forward_host(Mlp* m, const double* mu, int nmu, hipStream_t s) {
  RBWS_HIP(hipSetDevice(m->device));
  load_inputs(m, mu, nmu, s, nullptr);
  forward(m, nmu, false, s);
  return (const float*)m->o.ptr;
}

void mlp_predict_dev(Mlp* m, const double* mu, int nmu, const int* rows_dev, double* c, int cstride,
                     hipStream_t s) {
  if (nmu <= 0) return;
  RBWS_HIP(hipSetDevice(m->device));
  const double* md = nullptr;
  load_inputs(m, mu, nmu, s, &md);
  forward(m, nmu, false, s);
  hipLaunchKernelGGL(k_mlp_outc, dim3(blocks_for((long long)nmu * m->d.nout)), dim3(256), 0, s,
                     (const float*)m->o.ptr, nmu, m->outp[m->L - 1], m->d.nout, rows_dev, md, in_scale(m),
                     (const double*)m->scal.ptr, c, cstride);
  RBWS_HIP(hipGetLastError());
}

// pairs -> device inputs (bf16, npairs x inp0) and scaled targets (float, npairs x outp)
struct PairBufs {
  DevBuf xa, ya, perm, loss, mu, c;
};
static PairBufs& pair_bufs() {
  static thread_local PairBufs& p = *new PairBufs();
  return p;
}

static void load_pairs(Mlp* m, const double* mu, const double* c, int n, hipStream_t s) {
  check_mu(m, mu, n);
  RBWS_REQUIRE(c != nullptr, RBWS_EINVAL, "c is NULL");
  for (long long i = 0; i < (long long)n * m->d.nout; i++) RBWS_REQUIRE(std::isfinite(c[i]), RBWS_EINVAL, "c must be finite");
  PairBufs& P = pair_bufs();
  const int dev = m->device;
  const double* md = upload_d(P.mu, mu, (long long)n * m->d.p, dev, s);
  const double* cd = upload_d(P.c, c, (long long)n * m->d.nout, dev, s);
  const int K0 = m->inp[0], NO = m->outp[m->L - 1];
  __bf16* xa = (__bf16*)P.xa.get(sizeof(__bf16) * (long long)n * K0, dev);
  float* ya = (float*)P.ya.get(sizeof(float) * (long long)n * NO, dev);
  hipLaunchKernelGGL(k_mlp_in, dim3(blocks_for((long long)n * K0)), dim3(256), 0, s, md, n, n, K0, in_scale(m), xa);
  hipLaunchKernelGGL(k_mlp_tgt, dim3(blocks_for((long long)n * NO)), dim3(256), 0, s, md, cd, n, m->d.nout, NO,
                     in_scale(m), (const double*)m->scal.ptr, ya);
  RBWS_HIP(hipGetLastError());
}

// one training step's launches (gather, forward, loss, backward, optional Adam, tick)
static void step_launches(Mlp* m, int npairs, int nb, int t0, int hist, bool update, hipStream_t s) {
  PairBufs& P = pair_bufs();
  const AdamDev* ad = (const AdamDev*)m->ad.ptr;
  hipLaunchKernelGGL(k_mlp_gather, dim3(m->cap), dim3(64), 0, s, ad, t0, (const int*)P.perm.ptr, npairs, nb, m->cap,
                     (const __bf16*)P.xa.ptr, m->inp[0], (const float*)P.ya.ptr, m->outp[m->L - 1],
                     (__bf16*)m->x.ptr, (__bf16*)m->xt.ptr, (float*)m->c.ptr);
  forward(m, nb, true, s);
  backward(m, nb, ad, t0, hist, (double*)P.loss.ptr, s);
  if (update) {
    adam_all(m, t0, 1, s);
    hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(64), 0, s, (AdamDev*)m->ad.ptr);
  }
  RBWS_HIP(hipGetLastError());
}

static void set_schedule(Mlp* m, int T, int spe, double lr0, double lr_min, hipStream_t s) {
  AdamDev a;
  RBWS_HIP(hipMemcpyAsync(&a, m->ad.ptr, sizeof a, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  a.T = T;
  a.spe = spe;
  a.lr0 = lr0;
  a.lr_min = lr_min;
  RBWS_HIP(hipMemcpyAsync(m->ad.ptr, &a, sizeof a, hipMemcpyHostToDevice, s));
}

// single minibatch: gradients (update = false) or one Adam step
static double one_step(Mlp* m, const double* mu, const double* c, int nb, bool update, double lr, hipStream_t s) {
  RBWS_REQUIRE(nb >= 1, RBWS_EINVAL, "empty minibatch");
  RBWS_REQUIRE(std::isfinite(lr) && lr >= 0.0, RBWS_EINVAL, "bad step size");
  RBWS_HIP(hipSetDevice(m->device));
  load_pairs(m, mu, c, nb, s);
  ensure_ws(m, nb);
  PairBufs& P = pair_bufs();
  std::vector<int> id(nb);
  for (int i = 0; i < nb; i++) id[i] = i;
  RBWS_HIP(hipMemcpyAsync(P.perm.get(sizeof(int) * nb, m->device), id.data(), sizeof(int) * nb,
                          hipMemcpyHostToDevice, s));
  P.loss.get(sizeof(double), m->device);
  const AdamDev a0 = adam_host(m);
  set_schedule(m, 0, 1, lr, lr, s);
  step_launches(m, nb, nb, a0.t, 0, update, s);
  double loss = 0.0;
  RBWS_HIP(hipMemcpyAsync(&loss, P.loss.ptr, sizeof loss, hipMemcpyDeviceToHost, s));
  RBWS_HIP(hipStreamSynchronize(s));
  return loss;
}

double mlp_grad(Mlp* m, const double* mu, const double* c, int nb, float* grads, hipStream_t s) {
  const double loss = one_step(m, mu, c, nb, false, 0.0, s);
  if (grads) {
    std::vector<float> pad(m->npad);
    RBWS_HIP(hipMemcpyAsync(pad.data(), m->g.ptr, sizeof(float) * m->npad, hipMemcpyDeviceToHost, s));
    RBWS_HIP(hipStreamSynchronize(s));
    padded_to_pack(m, pad, grads);
  }
  return loss;
}

double mlp_adam_step(Mlp* m, const double* mu, const double* c, int nb, double lr, hipStream_t s) {
  return one_step(m, mu, c, nb, true, lr, s);
}

void mlp_train(Mlp* m, const double* mu, const double* c, int npairs, const rbws_mlp_train_cfg* cfg,
               double* loss_hist, hipStream_t s) {
  RBWS_REQUIRE(cfg != nullptr, RBWS_EINVAL, "cfg is NULL");
  RBWS_REQUIRE(cfg->epochs >= 1, RBWS_EINVAL, "epochs < 1");
  RBWS_REQUIRE(cfg->batch >= 1 && cfg->batch <= npairs, RBWS_EINVAL, "batch must be in 1..npairs");
  RBWS_REQUIRE(std::isfinite(cfg->lr) && cfg->lr > 0.0 && std::isfinite(cfg->lr_min) && cfg->lr_min >= 0.0,
               RBWS_EINVAL, "bad step sizes");
  RBWS_HIP(hipSetDevice(m->device));
  const int nb = cfg->batch, spe = npairs / nb, E = cfg->epochs;
  const long long T = (long long)E * spe;
  RBWS_REQUIRE(T < (1LL << 30), RBWS_EINVAL, "too many steps");
  load_pairs(m, mu, c, npairs, s);
  ensure_ws(m, nb);
  PairBufs& P = pair_bufs();
  // a seeded shuffle per epoch (Fisher-Yates on splitmix64)
  std::vector<int> perm((size_t)E * npairs);
  uint64_t st = cfg->seed;
  for (int e = 0; e < E; e++) {
    int* q = perm.data() + (size_t)e * npairs;
    for (int i = 0; i < npairs; i++) q[i] = i;
    for (int i = npairs - 1; i > 0; i--) {
      const int j = (int)(splitmix64(st) % (uint64_t)(i + 1));
      std::swap(q[i], q[j]);
    }
  }
  RBWS_HIP(hipMemcpyAsync(P.perm.get(sizeof(int) * perm.size(), m->device), perm.data(), sizeof(int) * perm.size(),
                          hipMemcpyHostToDevice, s));
  double* lossd = (double*)P.loss.get(sizeof(double) * T, m->device);
  const AdamDev a0 = adam_host(m);
  set_schedule(m, (int)T, spe, cfg->lr, cfg->lr_min, s);
  RBWS_HIP(hipStreamSynchronize(s));
  if (cfg->use_graph) {
    if (!m->own) RBWS_HIP(hipStreamCreateWithFlags(&m->own, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    RBWS_HIP(hipStreamBeginCapture(m->own, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < spe; k++) step_launches(m, npairs, nb, a0.t, 1, true, m->own);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(m->own, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    RBWS_HIP(hipStreamEndCapture(m->own, &graph));
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      RBWS_HIP(e);
    }
    for (int ep = 0; ep < E && e == hipSuccess; ep++) e = hipGraphLaunch(exec, m->own);
    if (e == hipSuccess) e = hipStreamSynchronize(m->own);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    RBWS_HIP(e);
  } else {
    for (long long k = 0; k < T; k++) step_launches(m, npairs, nb, a0.t, 1, true, s);
    RBWS_HIP(hipStreamSynchronize(s));
  }
  if (loss_hist) {
    RBWS_HIP(hipMemcpyAsync(loss_hist, lossd, sizeof(double) * T, hipMemcpyDeviceToHost, s));
    RBWS_HIP(hipStreamSynchronize(s));
  }
}

// ---------------------------------------------------------------------------
// checkpoint
// ---------------------------------------------------------------------------
static const char kMlpMagic[8] = {'R', 'B', 'W', 'S', 'M', 'L', 'P', '1'};

void mlp_save(const Mlp* m, const char* path) {
  RBWS_REQUIRE(path != nullptr, RBWS_EINVAL, "path is NULL");
  std::vector<float> p(m->np);
  mlp_get_params(m, p.data(), nullptr);
  FILE* f = std::fopen(path, "wb");
  RBWS_REQUIRE(f != nullptr, RBWS_EINVAL, std::string("cannot open ") + path);
  bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8;
  ok = ok && std::fwrite(&m->d, sizeof m->d, 1, f) == 1;
  ok = ok && std::fwrite(&m->np, sizeof m->np, 1, f) == 1;
  ok = ok && std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  ok = ok && std::fwrite(m->out_mean.data(), sizeof(double), m->d.nout, f) == (size_t)m->d.nout;
  ok = ok && std::fwrite(m->out_std.data(), sizeof(double), m->d.nout, f) == (size_t)m->d.nout;
  ok = (std::fclose(f) == 0) && ok;
  RBWS_REQUIRE(ok, RBWS_EINVAL, std::string("writing ") + path + " failed");
}

Mlp* mlp_load(const char* path, int device) {
  RBWS_REQUIRE(path != nullptr, RBWS_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "rb");
  RBWS_REQUIRE(f != nullptr, RBWS_EINVAL, std::string("cannot open ") + path);
  char mag[8];
  rbws_mlp_desc d;
  long long np = 0;
  bool ok = std::fread(mag, 1, 8, f) == 8 && std::memcmp(mag, kMlpMagic, 8) == 0;
  ok = ok && std::fread(&d, sizeof d, 1, f) == 1;
  ok = ok && std::fread(&np, sizeof np, 1, f) == 1 && np > 0 && np < (1LL << 31);
  std::vector<float> p;
  std::vector<double> mean, sd;
  if (ok) {
    p.resize(np);
    ok = std::fread(p.data(), sizeof(float), np, f) == (size_t)np;
  }
  if (ok && d.nout >= 1 && d.nout <= 64) {
    mean.resize(d.nout);
    sd.resize(d.nout);
    ok = std::fread(mean.data(), sizeof(double), d.nout, f) == (size_t)d.nout &&
         std::fread(sd.data(), sizeof(double), d.nout, f) == (size_t)d.nout;
  } else {
    ok = false;
  }
  std::fclose(f);
  RBWS_REQUIRE(ok, RBWS_EINVAL, std::string("not a network checkpoint: ") + path);
  Mlp* m = mlp_create(&d, device, nullptr, 0);
  try {
    RBWS_REQUIRE(m->np == np, RBWS_EINVAL, "checkpoint size mismatch");
    mlp_set_params(m, p.data(), nullptr);
    mlp_set_scaling(m, mean.data(), sd.data(), nullptr);
  } catch (...) {
    mlp_destroy(m);
    throw;
  }
  return m;
}

}  // namespace rbws
