// rbws_internal.hpp -- shared declarations of the HIP library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rbws.h"

namespace rbws {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
  rbws_status code;
  std::string msg;
};
#define RBWS_HIP(expr)                                                               \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::rbws::Error{RBWS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define RBWS_REQUIRE(cond, code, msg)                 \
  do {                                                \
    if (!(cond)) throw ::rbws::Error{code, (msg)};    \
  } while (0)

// ---------------------------------------------------------------------------
// grid and face-class tables
//
// Scaled integer coordinates: node i -> 20 i, face between i and i+1 ->
// 10 (2i+1), a sub-domain boundary at t tenths -> 2 (n+1) t (unit cube
// scaled by 20 (n+1)).  Along each axis the breakpoints split the line into
// open intervals; a position gets the code 2m (inside interval m) or 2m+1
// (on breakpoint m).  Codes that occur on a given grid are renumbered
// densely.  A face class is the triple of its three axis codes; the
// coefficient of a class is the mean over the 2^t corners obtained by
// nudging every on-breakpoint coordinate to both sides (t = number of such
// coordinates), summed pairwise in corner order and scaled by 2^-t.
// ---------------------------------------------------------------------------
constexpr int kMaxClass = 4096;
constexpr int kMaxQ = 32;

struct GridDev {
  int n;
  long long ndof;
  const uint8_t* code[3][2];  // [axis][0 = node (index i-1), 1 = face (index i)]
  int ncode[3];               // dense codes per axis
  int nclass;                 // ncode[0]*ncode[1]*ncode[2]
  int ndir;                   // 1 (isotropic) or 3 (one table per face direction)
};

// per-class corner table: theta index of each corner (up to 8), per direction
struct ClassTable {
  int nclass, ndir;
  std::vector<uint8_t> ncorner;     // [nclass] = 2^t
  std::vector<uint8_t> theta_idx;   // [ndir][nclass][8]
};

struct Problem {
  rbws_problem_desc desc;
  std::vector<int> blocks;
  int device;
  int n, p, Q;
  long long ndof;
  GridDev grid;        // device pointers into `codes_dev`
  uint8_t* codes_dev;  // 6 code arrays
  ClassTable ct;
  uint8_t* ct_ncorner_dev;
  uint8_t* ct_theta_dev;
};

// ---------------------------------------------------------------------------
// per-solve CG state (device memory)
// ---------------------------------------------------------------------------
enum SolveMode : int { MODE_RESID = 0, MODE_ITER = 1, MODE_DONE = 2 };

struct CgState {
  double rho, alpha, beta, rr, thr, ff, init_rr, tol2;
  int k, extra, status, mode, restart, skip2, maxit, prec, first, mg;  // mg: P is a V-cycle
  int nvc;                                                             // V-cycles applied
  unsigned long long t_done;
};

// ---------------------------------------------------------------------------
// small host helpers
// ---------------------------------------------------------------------------
inline int p_of(const rbws_problem_desc& d) {
  if (d.kind == RBWS_KIND_BLOCKS) return d.nblocks;
  if (d.kind == RBWS_KIND_OCTANTS) return 8;
  return 24 + (d.f_kind == RBWS_F_GAUSS ? 3 : 0);
}
inline int q_of(const rbws_problem_desc& d) {
  if (d.kind == RBWS_KIND_BLOCKS) return d.nblocks + 1;
  if (d.kind == RBWS_KIND_OCTANTS) return 8;
  return 24;
}
void theta_host(const Problem& P, const double* mu, double* theta);

}  // namespace rbws
