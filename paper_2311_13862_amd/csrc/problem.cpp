// problem.cpp -- host side of the operator setup: grid codes and face classes.
//
// The coefficient kappa(mu) is piecewise constant on axis-aligned boxes (the
// paper's Example 2 uses such sub-domains, Sec. 4).  Instead of storing 3 n^3
// face coefficients per parameter, the library stores O(n) bytes of codes per
// axis and a table of face classes; a class's coefficient for any theta is
// the mean over its corners of theta[corner's affine term].  Per parameter
// only the class table (<= a few thousand values) is materialised, so the
// stencil reads 0 bytes of coefficients per unknown from HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "rbws_internal.hpp"

namespace rbws {

namespace {

// sorted unique breakpoints (scaled coordinates) along an axis
std::vector<long> breakpoints(const rbws_problem_desc& d, const std::vector<int>& blocks, int axis) {
  std::vector<long> b;
  long s = 2L * (d.n + 1);
  if (d.kind == RBWS_KIND_BLOCKS) {
    for (int k = 0; k < d.nblocks; k++) {
      b.push_back(s * blocks[6 * k + 2 * axis]);
      b.push_back(s * blocks[6 * k + 2 * axis + 1]);
    }
  } else {
    b.push_back(10L * (d.n + 1));
  }
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end()), b.end());
  return b;
}

int raw_code(const std::vector<long>& bp, long X) {
  int m = (int)(std::lower_bound(bp.begin(), bp.end(), X) - bp.begin());
  if (m < (int)bp.size() && bp[m] == X) return 2 * m + 1;
  return 2 * m;
}

// a representative coordinate (doubled units) strictly inside interval m
double interval_rep(const std::vector<long>& bp, int m) {
  int L = (int)bp.size();
  if (m == 0) return 2.0 * bp[0] - 1.0;
  if (m == L) return 2.0 * bp[L - 1] + 1.0;
  return (double)(bp[m - 1] + bp[m]);
}

}  // namespace

void build_tables(Problem& P) {
  const rbws_problem_desc& d = P.desc;
  const int n = d.n;
  std::vector<long> bp[3];
  std::vector<int> raw[3][2];          // raw codes of nodes / faces per axis
  std::vector<int> dense_of_raw[3];    // raw code -> dense code (-1 unused)
  std::vector<int> raw_of_dense[3];
  for (int a = 0; a < 3; a++) {
    bp[a] = breakpoints(d, P.blocks, a);
    raw[a][0].resize(n);
    raw[a][1].resize(n + 1);
    for (int i = 1; i <= n; i++) raw[a][0][i - 1] = raw_code(bp[a], 20L * i);
    for (int i = 0; i <= n; i++) raw[a][1][i] = raw_code(bp[a], 10L * (2 * i + 1));
    int nraw = 2 * (int)bp[a].size() + 1;
    std::vector<char> used(nraw, 0);
    for (int t = 0; t < 2; t++)
      for (int c : raw[a][t]) used[c] = 1;
    dense_of_raw[a].assign(nraw, -1);
    for (int c = 0; c < nraw; c++)
      if (used[c]) {
        dense_of_raw[a][c] = (int)raw_of_dense[a].size();
        raw_of_dense[a].push_back(c);
      }
    P.grid.ncode[a] = (int)raw_of_dense[a].size();
  }
  const int N0 = P.grid.ncode[0], N1 = P.grid.ncode[1], N2 = P.grid.ncode[2];
  const int nclass = N0 * N1 * N2;
  RBWS_REQUIRE(nclass <= kMaxClass, RBWS_EINVAL, "too many face classes for this sub-domain layout");
  const int ndir = d.kind == RBWS_KIND_OCTANTS_ANISO ? 3 : 1;
  RBWS_REQUIRE(ndir * nclass <= kMaxClass, RBWS_EINVAL, "too many face classes for this sub-domain layout");
  P.grid.nclass = nclass;
  P.grid.ndir = ndir;
  P.ct.nclass = nclass;
  P.ct.ndir = ndir;
  P.ct.ncorner.assign(nclass, 1);
  P.ct.theta_idx.assign((size_t)ndir * nclass * 8, 0);

  const long s = 2L * (n + 1);
  for (int c0 = 0; c0 < N0; c0++)
    for (int c1 = 0; c1 < N1; c1++)
      for (int c2 = 0; c2 < N2; c2++) {
        const int cls = (c0 * N1 + c1) * N2 + c2;
        const int rc[3] = {raw_of_dense[0][c0], raw_of_dense[1][c1], raw_of_dense[2][c2]};
        int tied[3], t = 0;
        for (int a = 0; a < 3; a++)
          if (rc[a] & 1) tied[t++] = a;
        const int nc = 1 << t;
        P.ct.ncorner[cls] = (uint8_t)nc;
        for (int corner = 0; corner < nc; corner++) {
          // interval code per axis: untied keep theirs; tied go to the lower
          // (bit 0) or upper (bit 1) neighbour interval; the first tied axis
          // is the most significant bit of the corner index
          int iv[3] = {rc[0], rc[1], rc[2]};
          for (int m = 0; m < t; m++) {
            int up = (corner >> (t - 1 - m)) & 1;
            iv[tied[m]] = up ? rc[tied[m]] + 1 : rc[tied[m]] - 1;
          }
          double rep[3];
          for (int a = 0; a < 3; a++) rep[a] = interval_rep(bp[a], iv[a] / 2);
          int region = 0;
          if (d.kind == RBWS_KIND_BLOCKS) {
            for (int b = d.nblocks - 1; b >= 0; b--) {
              const int* B = &P.blocks[6 * b];
              bool in = true;
              for (int a = 0; a < 3; a++) {
                double lo = 2.0 * s * B[2 * a], hi = 2.0 * s * B[2 * a + 1];
                if (!(rep[a] > lo && rep[a] < hi)) in = false;
              }
              if (in) { region = b + 1; break; }
            }
          } else {
            double mid = 2.0 * 10.0 * (n + 1);
            for (int a = 0; a < 3; a++)
              if (rep[a] > mid) region |= 1 << a;
          }
          for (int dir = 0; dir < ndir; dir++) {
            int idx = ndir == 3 ? 3 * region + dir : region;
            P.ct.theta_idx[((size_t)dir * nclass + cls) * 8 + corner] = (uint8_t)idx;
          }
        }
      }

  // device copies: dense codes of nodes and faces per axis, and the class table
  std::vector<uint8_t> codes;
  size_t off[3][2];
  for (int a = 0; a < 3; a++)
    for (int t = 0; t < 2; t++) {
      off[a][t] = codes.size();
      for (int c : raw[a][t]) codes.push_back((uint8_t)dense_of_raw[a][c]);
    }
  RBWS_HIP(hipSetDevice(P.device));
  RBWS_HIP(hipMalloc(&P.codes_dev, codes.size()));
  RBWS_HIP(hipMemcpy(P.codes_dev, codes.data(), codes.size(), hipMemcpyHostToDevice));
  for (int a = 0; a < 3; a++)
    for (int t = 0; t < 2; t++) P.grid.code[a][t] = P.codes_dev + off[a][t];
  RBWS_HIP(hipMalloc(&P.ct_ncorner_dev, P.ct.ncorner.size()));
  RBWS_HIP(hipMemcpy(P.ct_ncorner_dev, P.ct.ncorner.data(), P.ct.ncorner.size(), hipMemcpyHostToDevice));
  RBWS_HIP(hipMalloc(&P.ct_theta_dev, P.ct.theta_idx.size()));
  RBWS_HIP(hipMemcpy(P.ct_theta_dev, P.ct.theta_idx.data(), P.ct.theta_idx.size(), hipMemcpyHostToDevice));
  P.grid.n = n;
  P.grid.ndof = P.ndof;
}

void theta_host(const Problem& P, const double* mu, double* theta) {
  if (P.desc.kind == RBWS_KIND_BLOCKS) {
    theta[0] = 1.0;
    for (int b = 0; b < P.desc.nblocks; b++) theta[b + 1] = mu[b];
  } else {
    for (int q = 0; q < P.Q; q++) theta[q] = mu[q];
  }
}

Problem* problem_create(const rbws_problem_desc* d, int device) {
  RBWS_REQUIRE(d != nullptr, RBWS_EINVAL, "desc is NULL");
  RBWS_REQUIRE(d->n >= 1 && d->n <= 1024, RBWS_EINVAL, "n must be in [1, 1024]");
  RBWS_REQUIRE(d->kind >= 0 && d->kind <= 2, RBWS_EINVAL, "unknown problem kind");
  RBWS_REQUIRE(d->f_kind == RBWS_F_ONE || d->f_kind == RBWS_F_GAUSS, RBWS_EINVAL, "unknown f kind");
  RBWS_REQUIRE(d->f_kind == RBWS_F_ONE || d->kind == RBWS_KIND_OCTANTS_ANISO, RBWS_EINVAL,
               "the Gaussian source needs the anisotropic octant kind");
  if (d->f_kind == RBWS_F_GAUSS)
    RBWS_REQUIRE(d->gauss_width >= 0.005, RBWS_EINVAL,
                 "gauss_width must be at least 0.005 (exponents stay above -700 on the unit cube)");
  if (d->kind == RBWS_KIND_BLOCKS) {
    RBWS_REQUIRE(d->nblocks >= 1 && d->nblocks < kMaxQ, RBWS_EINVAL, "nblocks out of range");
    RBWS_REQUIRE(d->blocks != nullptr, RBWS_EINVAL, "blocks is NULL");
    for (int i = 0; i < 6 * d->nblocks; i++)
      RBWS_REQUIRE(d->blocks[i] >= 0 && d->blocks[i] <= 10, RBWS_EINVAL, "block bounds must be tenths 0..10");
    for (int b = 0; b < d->nblocks; b++)
      for (int a = 0; a < 3; a++)
        RBWS_REQUIRE(d->blocks[6 * b + 2 * a] < d->blocks[6 * b + 2 * a + 1], RBWS_EINVAL,
                     "block lower bound must be below upper bound");
  }
  int ndev = 0;
  RBWS_HIP(hipGetDeviceCount(&ndev));
  RBWS_REQUIRE(device >= 0 && device < ndev, RBWS_EINVAL, "invalid device ordinal");
  Problem* P = new Problem();
  P->desc = *d;
  if (d->kind == RBWS_KIND_BLOCKS) P->blocks.assign(d->blocks, d->blocks + 6 * d->nblocks);
  P->desc.blocks = nullptr;
  P->device = device;
  P->n = d->n;
  P->p = p_of(*d);
  P->Q = q_of(*d);
  P->ndof = (long long)d->n * d->n * d->n;
  P->codes_dev = nullptr;
  P->ct_ncorner_dev = nullptr;
  P->ct_theta_dev = nullptr;
  try {
    build_tables(*P);
  } catch (...) {
    if (P->codes_dev) (void)hipFree(P->codes_dev);
    if (P->ct_ncorner_dev) (void)hipFree(P->ct_ncorner_dev);
    if (P->ct_theta_dev) (void)hipFree(P->ct_theta_dev);
    delete P;
    throw;
  }
  return P;
}

void problem_destroy(Problem* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  if (P->codes_dev) (void)hipFree(P->codes_dev);
  if (P->ct_ncorner_dev) (void)hipFree(P->ct_ncorner_dev);
  if (P->ct_theta_dev) (void)hipFree(P->ct_theta_dev);
  delete P;
}

}  // namespace rbws
