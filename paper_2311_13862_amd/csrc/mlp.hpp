// mlp.hpp -- the learned start: a multilayer perceptron trained and evaluated
// on the BF16 matrix cores (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "solver.hpp"

namespace rbws {

// step counter and step-size schedule (device memory, read by the kernels so
// that a captured training epoch can be replayed without host updates)
struct AdamDev {
  int t;      // completed steps
  int T;      // steps of the cosine schedule (0: constant lr0)
  int spe;    // steps per epoch (minibatch position = t % spe)
  int pad;
  double lr0, lr_min, b1, b2, eps;
};

struct Mlp {
  int device = 0;
  rbws_mlp_desc d{};
  int L = 0;                          // weight layers: depth hidden + 1 output
  std::vector<int> in, out, inp, outp;  // real and padded (multiple of 32) sizes
  std::vector<long long> wo, bo;      // offsets of W_l and b_l in the padded FP32 arrays
  std::vector<long long> wbo, wto;    // offsets of W_l (outp x inp) and W_l^T in the BF16 arrays
  long long np = 0;                   // packed (unpadded) parameter count
  long long npad = 0, nbf = 0;
  int maxw = 0;                       // widest padded layer
  DevBuf w, m, v, g;                  // FP32 master weights, Adam moments, gradients
  DevBuf wb, wt;                      // BF16 W and W^T
  DevBuf ad;                          // AdamDev
  DevBuf scal;                        // out_mean[nout], out_std[nout] (double)
  std::vector<double> out_mean, out_std;
  // workspace for up to `cap` rows
  int cap = 0;
  DevBuf x, xt, c, o, zs, hs, hts, g32, gb, gt, loss;
  hipStream_t own = nullptr;          // stream of captured training graphs

  long long z_off(int l) const { return (long long)l * cap * maxw; }
};

Mlp* mlp_create(const rbws_mlp_desc* d, int device, const float* params, unsigned long long seed);
void mlp_destroy(Mlp* m);
void mlp_set_params(Mlp* m, const float* params, hipStream_t s);
void mlp_get_params(const Mlp* m, float* params, hipStream_t s);
void mlp_set_scaling(Mlp* m, const double* mean, const double* stdev, hipStream_t s);
void mlp_fit_scaling(Mlp* m, const double* mu, const double* c, int npairs, hipStream_t s);
// raw network outputs y (device, nmu x outp[L-1] floats) for host mu
const float* mlp_forward_host(Mlp* m, const double* mu, int nmu, hipStream_t s);
// c (device, nmu rows of stride cstride, double) for host mu (rows `rows` of the
// batch, or 0..nmu-1 when rows is null)
void mlp_predict_dev(Mlp* m, const double* mu, int nmu, const int* rows_dev, double* c, int cstride,
                     hipStream_t s);
double mlp_grad(Mlp* m, const double* mu, const double* c, int nb, float* grads, hipStream_t s);
double mlp_adam_step(Mlp* m, const double* mu, const double* c, int nb, double lr, hipStream_t s);
void mlp_train(Mlp* m, const double* mu, const double* c, int npairs, const rbws_mlp_train_cfg* cfg,
               double* loss_hist, hipStream_t s);
void mlp_save(const Mlp* m, const char* path);
Mlp* mlp_load(const char* path, int device);

}  // namespace rbws
