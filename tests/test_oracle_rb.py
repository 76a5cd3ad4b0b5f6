"""Pins for the oracle's reduced basis: greedy build (Alg. 4 skeleton),
Galerkin online solve (Eq. "RB system") and the warm-started solve (Alg. 5).

Checked against: orthonormality of V; the Galerkin property that any vector
in span V is reproduced exactly (so every greedy snapshot is recovered by the
RB solve at its own parameter); symmetry and Galerkin-orthogonality of the
reduced system; numpy's dense Cholesky/solve and matrix products; the scaling
c(2 mu) = c(mu)/2 of the octant problem; and the paper's empirical claim that
warm-started solves need no more iterations than zero-started ones on the
16^3 three-block problem (Sec. 4, Tables 1-2).
"""
import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W


@pytest.fixture(scope="module")
def c1():
    wl = W.blocks3_16()
    P = oracle.Problem(wl.problem)
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    B = oracle.greedy(P, mut, wl.N, wl.snap_tol, prec=oracle.PREC_JACOBI)
    return wl, P, mut, B


def test_basis_orthonormal(c1):
    wl, P, mut, B = c1
    assert B.N == wl.N
    assert np.abs(B.V @ B.V.T - np.eye(B.N)).max() <= 1e-13
    assert B.selected[0] == 0 and len(set(B.selected.tolist())) == B.N


def test_selection_is_argmax(c1):
    wl, P, mut, B = c1
    for k in range(B.N - 1):
        row = B.hist[k]
        assert B.selected[k + 1] == int(np.argmax(row))       # first maximal index


def test_reduced_matrices(c1):
    wl, P, mut, B = c1
    N = B.N
    for q in range(P.Q):
        e = np.zeros(P.Q)
        e[q] = 1.0
        AqV = np.stack([P.apply_theta(e, v) for v in B.V])
        ref = B.V @ AqV.T
        assert np.array_equal(B.AqN[q, :N, :N], B.AqN[q, :N, :N].T)
        np.testing.assert_allclose(B.AqN[q, :N, :N], ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    f = P.rhs(mut[0])
    np.testing.assert_allclose(B.fN[:N], B.V @ f, rtol=0, atol=1e-15 * np.abs(B.fN).max())


def test_online_solve_vs_numpy(c1):
    wl, P, mut, B = c1
    N = B.N
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 8, W.SEED_TEST)
    for m in mus:
        th = P.theta(m)
        AN = np.tensordot(th, B.AqN[:, :N, :N], axes=1)
        np.linalg.cholesky(AN)
        c = B.coeffs(m)
        np.testing.assert_allclose(c, np.linalg.solve(AN, B.fN[:N]), rtol=0,
                                   atol=1e-12 * np.abs(c).max())
        u0 = B.lift(c)
        np.testing.assert_allclose(u0, B.V.T @ c, rtol=0, atol=1e-15 * np.abs(u0).max())
        # Galerkin orthogonality: V^T (f - A V c) = 0 up to rounding
        r0 = P.rhs(m) - P.apply(m, u0)
        assert np.linalg.norm(B.V @ r0) <= 1e-12 * np.linalg.norm(P.rhs(m))


def test_snapshots_reproduced(c1):
    wl, P, mut, B = c1
    for l in B.selected:
        m = mut[l]
        u, st = P.cg(m, prec=oracle.PREC_JACOBI, tol=wl.snap_tol)
        urb = B.lift(B.coeffs(m))
        assert np.linalg.norm(urb - u) <= 1e-10 * np.linalg.norm(u)
        f = P.rhs(m)
        r = f - P.apply(m, urb)
        assert np.linalg.norm(r) <= 10 * wl.snap_tol * np.linalg.norm(f)
    # the indicator at the selected parameters is tiny, at others it is not
    last = B.hist[-1]
    assert last[B.selected].max() <= 10 * wl.snap_tol
    assert np.median(last) > 1e3 * wl.snap_tol


def test_warm_start_not_worse(c1):
    wl, P, mut, B = c1
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    for prec in (oracle.PREC_NONE, oracle.PREC_JACOBI):
        z = [P.cg(m, prec=prec, tol=wl.tol)[1]["iters"] for m in mus]
        w = [oracle.rbi_cg(B, m, prec=prec, tol=wl.tol)[1]["iters"] for m in mus]
        assert max(np.subtract(w, z)) <= 0
        assert np.mean(w) < np.mean(z)


def test_octant_coefficient_scaling():
    spec = W.Problem(6, W.KIND_OCTANTS)
    P = oracle.Problem(spec)
    mut = W.sample_mu(spec, 0.01, 100.0, 24, W.SEED_TRAIN)
    B = oracle.greedy(P, mut, 6, 1e-12)
    for m in W.sample_mu(spec, 0.01, 100.0, 4, W.SEED_TEST):
        c1, c2 = B.coeffs(m), B.coeffs(2.0 * m)
        np.testing.assert_allclose(c2, c1 / 2, rtol=1e-14, atol=1e-16 * np.abs(c1).max())


def test_chol_breakdown_reported():
    spec = W.Problem(4, W.KIND_OCTANTS)
    P = oracle.Problem(spec)
    mut = W.sample_mu(spec, 0.1, 10.0, 8, W.SEED_TRAIN)
    B = oracle.greedy(P, mut, 3, 1e-12)
    with pytest.raises(FloatingPointError):
        B.coeffs(-np.ones(8))
