"""Seeded synthetic workloads: problem descriptions and parameter samples.

This module is shared by the HIP path's callers and by the test/benchmark
code that drives the CPU oracle.  It holds *data only*: grid sizes, the
axis-aligned blocks (in tenths of the unit cube) on which the diffusion
coefficient is piecewise constant, the parameter ranges and the seeded
samplers.  None of the method's arithmetic (face coefficients, operators,
solvers, reduced bases) lives here.

The shapes follow the paper's 3D diffusion tests (Sec. 4, Examples 1-2):
a parametrized coefficient that is piecewise constant on sub-boxes, a
many-query test set, and a greedy training set.  The paper's finite-element
discretisation is replaced by 7-point finite differences on interior grids
of n^3 points with zero Dirichlet data.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

# problem kinds (mirror the C enum in include/rbws.h)
KIND_BLOCKS = 0          # kappa = 1 + sum over blocks, painter's order, isotropic
KIND_OCTANTS = 1         # kappa = mu_q on octant q (2x2x2 split at 0.5), isotropic
KIND_OCTANTS_ANISO = 2   # (kx, ky, kz) per octant, 24 parameters

F_ONE = 0                # f = 1
F_GAUSS = 1              # f = exp(-|x - x0(mu)|^2 / width), x0 = mu[24:27]

# seeds for the samplers
SEED_TRAIN = 0
SEED_TEST = 1
SEED_MLP_PAIRS = 2
SEED_MLP_INIT = 3

BLOCKS3 = ((1, 4, 1, 4, 1, 4),
           (6, 9, 1, 4, 6, 9),
           (3, 7, 3, 7, 3, 7))
BLOCKS4 = BLOCKS3 + ((1, 3, 7, 9, 1, 3),)


@dataclasses.dataclass(frozen=True)
class Problem:
    """Description of one parametrized operator family A_h(mu), f_h(mu)."""
    n: int                                   # interior points per axis
    kind: int = KIND_BLOCKS
    blocks: Tuple[Tuple[int, ...], ...] = ()  # (xlo,xhi,ylo,yhi,zlo,zhi) in tenths
    f_kind: int = F_ONE
    gauss_width: float = 0.02

    @property
    def p(self) -> int:
        if self.kind == KIND_BLOCKS:
            return len(self.blocks)
        if self.kind == KIND_OCTANTS:
            return 8
        return 24 + (3 if self.f_kind == F_GAUSS else 0)

    @property
    def Q(self) -> int:
        """Number of affine terms theta_q(mu) A_q."""
        if self.kind == KIND_BLOCKS:
            return len(self.blocks) + 1
        if self.kind == KIND_OCTANTS:
            return 8
        return 24

    @property
    def ndof(self) -> int:
        return self.n ** 3

    def blocks_flat(self) -> np.ndarray:
        return np.asarray(self.blocks, dtype=np.int32).reshape(-1)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    mu_lo: float
    mu_hi: float
    n_train: int
    N: int
    n_test: int
    tol: float
    snap_tol: float
    precision: str            # "fp64" or "fp32ir"
    n_mlp_pairs: int = 0


def sample_mu(problem: Problem, lo: float, hi: float, count: int, seed: int) -> np.ndarray:
    """(count, p) float64 parameters.

    Diffusion parameters are log-uniform in [lo, hi]; for the Gaussian source
    the last three entries are the centre x0, uniform in [0.25, 0.75].
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=(count, problem.p))
    a, b = np.log10(lo), np.log10(hi)
    mu = np.empty_like(u)
    nk = problem.p - (3 if problem.f_kind == F_GAUSS else 0)
    mu[:, :nk] = 10.0 ** (a + (b - a) * u[:, :nk])
    if problem.f_kind == F_GAUSS:
        mu[:, nk:] = 0.25 + 0.5 * u[:, nk:]
    return np.ascontiguousarray(mu)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
def blocks3_16() -> Workload:
    """16^3, three blocks, FP64, greedy N=20 from 256 training parameters."""
    return Workload("blocks3-16^3-fp64", Problem(16, KIND_BLOCKS, BLOCKS3),
                    0.1, 10.0, n_train=256, N=20, n_test=32, tol=1e-12,
                    snap_tol=1e-13, precision="fp64")


def blocks4_64() -> Workload:
    """64^3, four blocks, FP64 batched, N=30 from 512 training parameters."""
    return Workload("blocks4-64^3-fp64", Problem(64, KIND_BLOCKS, BLOCKS4),
                    0.1, 10.0, n_train=512, N=30, n_test=256, tol=1e-10,
                    snap_tol=1e-12, precision="fp64")


def octants_128() -> Workload:
    """128^3, 2x2x2 octants (p=8), FP32-in-FP64 refinement, N=40."""
    return Workload("octants8-128^3-fp32ir", Problem(128, KIND_OCTANTS),
                    0.01, 100.0, n_train=1024, N=40, n_test=1024, tol=1e-10,
                    snap_tol=1e-12, precision="fp32ir", n_mlp_pairs=8192)


def aniso_mixed(n: int) -> Workload:
    """Anisotropic octants + Gaussian source (p=27) at one grid size."""
    return Workload(f"aniso27-{n}^3-fp32ir",
                    Problem(n, KIND_OCTANTS_ANISO, (), F_GAUSS, 0.02),
                    0.1, 10.0, n_train=1024, N=60, n_test=512, tol=1e-10,
                    snap_tol=1e-12, precision="fp32ir", n_mlp_pairs=8192)


MIXED_SIZES = (64, 96, 128)


def mixed_assignment(count: int) -> np.ndarray:
    """Grid-size index of solve i in the uneven batch: i mod 3."""
    return np.arange(count, dtype=np.int32) % len(MIXED_SIZES)


def theta_len(problem: Problem) -> int:
    return problem.Q


def scaled(problem: Problem, n: Optional[int] = None) -> Problem:
    """Same operator family on another grid size."""
    return dataclasses.replace(problem, n=problem.n if n is None else n)
