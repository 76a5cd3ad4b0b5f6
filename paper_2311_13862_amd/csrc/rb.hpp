// rb.hpp -- reduced basis on the device: greedy build, online solve, lift.
#pragma once
#include <vector>

#include "solver.hpp"

namespace rbws {

struct Basis {
  const Problem* prob = nullptr;
  int Nmax = 0, N = 0, Q = 0;
  long long ndof = 0;
  DevBuf V;                  // Nmax x ndof, row j = basis vector j (orthonormal)
  std::vector<double> AqN;   // Q x Nmax x Nmax: A_q^N = V^T A_q V
  std::vector<double> fN;    // Nmax: V^T f (f = 1 only)
  DevBuf AqN_d, fN_d;        // device copies
  std::vector<int> selected;
  std::vector<double> hist;  // N x ntrain indicators (row k: k+1 basis vectors)
  int ntrain = 0;
  double final_max = 0.0;    // max over the training set of the final indicator
  // Residual decomposition for a fixed source f (built by rb_build when f = 1 and
  // the vectors W_(q,i) = A_q v_i fit in memory): with y_(q,i) = theta_q c_i,
  //   ||f - A(mu) V c||^2 = ff - 2 y^T g + y^T G y,
  // G_(q,i),(q',j) = W_(q,i)^T W_(q',j), g_(q,i) = W_(q,i)^T f, ff = f^T f
  // (correctly rounded dots); index (q, i) = q Nmax + i.
  bool est = false;
  double ff = 0.0;
  std::vector<double> G, g;
  DevBuf G_d, g_d;
  // kind 1: an L1ROC basis (Sec. 3.1, Alg. 4).  V holds the DEIM-normalised
  // vectors W; the online coefficients solve the collocation least-squares
  // problem at the points pts (ascending grid indices, snapshot points xs and
  // residual points xr merged); T (Nmax x Nmax, upper triangular) gives W = U T
  // with U the snapshots, for the L1 indicator.  AqN and fN are unused.
  int kind = 0;
  std::vector<long long> pts, xs, xr;
  std::vector<double> T;
  DevBuf pts_d, T_d;
  void upload(hipStream_t s);
};

// per-solve view of a basis for the online kernels
struct RbDev {
  const double* AqN;
  const double* fN;
  const double* V;
  int N, ld, Q, pad;
};

Basis* rb_build(const Problem* P, const double* mu_train, int ntrain, int N, double snap_tol,
                int prec, int snap_maxit, int flags, hipStream_t s);

// L1ROC greedy (Sec. 3.1, Alg. 4): snapshots by PCG, DEIM of each snapshot and
// of the current approximation's residual at the chosen parameter, the L1
// indicator over the training set; N <= kL1MaxN.
Basis* rb_build_l1roc(const Problem* P, const double* mu_train, int ntrain, int N, double snap_tol,
                      int prec, int snap_maxit, int flags, hipStream_t s);
constexpr int kL1MaxN = 60;

// ||f - A(mu_b) V c_b|| / ||f|| for every solve of B from the residual
// decomposition of its problem's basis (every basis must have `est`); c device,
// row b at b * cstride.  rel: host, nsolve values.  Returns the number of
// solves whose value is not trustworthy (the squared residual below 1e-8 of
// the magnitude of its terms, where cancellation could dominate).
int rb_resid_estimate(Batch& B, const std::vector<const Basis*>& bases, const double* c, int cstride, double* rel,
                      hipStream_t s);

// c (device, nsolve x cstride) for every solve of batch B from the bases of its
// problems (bases[prob]); theta comes from the batch.  Returns the number of
// solves whose reduced matrix was not positive definite.
int rb_coeffs(Batch& B, const std::vector<const Basis*>& bases, double* c, int cstride, int force_exact,
              hipStream_t s);

// u_b = V c_b (correctly rounded per entry) into the batch layout `u`
void rb_lift_exact(Batch& B, const std::vector<const Basis*>& bases, const double* c, int cstride,
                   double* u, int force_exact, hipStream_t s);

// u_b = V c_b with FP64 MFMA (single problem, all solves use bases[0])
void rb_lift_mfma(Batch& B, const Basis* basis, const double* c, int cstride, double* u, hipStream_t s);

void basis_save(const Basis* b, const char* path);
Basis* basis_load(const Problem* P, const char* path, hipStream_t s);

}  // namespace rbws
