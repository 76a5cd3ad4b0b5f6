// mg.hpp -- the multigrid V-cycle preconditioner (Alg. 2) for batched PCG.
#pragma once
#include <hip/hip_runtime.h>

#include "solver.hpp"

namespace rbws {

struct MgRun;

// Levels of a grid: n_0 = n, n_{l+1} = (n_l - 1) / 2 while n_l > 3.
int mg_levels_of(int n, int* out);

// Hierarchy for every solve of batch B: per problem of the batch, the coarse
// grids, each solve's face-coefficient tables on them, the transfer tables and
// the coarsest-level Cholesky factors.  fp32 selects the vector type of
// mg_apply.  The object is reused (and rebuilt) by the next call on this thread.
MgRun* mg_prepare(Batch& B, int nu, double omega, bool fp32, hipStream_t s);

// s_b = MG(r_b) (one V-cycle from zero) for every solve on the V-cycle lists
// of L (Lists::mg, filled by the per-solve finalisers); r and s are device
// vectors laid out like the batch (double or float).
// Returns true when the level-0 post-smoothing also wrote the r^T s partials
// of every listed tile (partial slot 1 in FP64, IrPart.g[2] in FP32).
bool mg_apply(MgRun* m, Batch& B, const void* r, void* s, const Lists& L, void* part, hipStream_t st);

// s_b = MG(r_b) for every solve of B, outside a solve: every tile and every
// solve listed, then one V-cycle.  Synchronises the stream.
void mg_apply_all(Batch& B, int nu, double omega, bool fp32, const void* r, void* s, hipStream_t st);

// Whether the FP32 post-smoothing of levels whose tiles span whole rows forms
// the z/y interpolation of the coarse correction itself (default) or reads it
// from a separate pass; applies from the next mg_prepare on.
bool mg_pz_enabled();
void set_mg_pz(int on);

}  // namespace rbws
