"""Pins for the oracle's multigrid preconditioner (Alg. 2) and MGCG (Alg. 1
with P = MG), against what mathematics and textbook routines fix:

- every entry of the restriction and prolongation equals the dense Kronecker
  form scale P^T r and P e (P from numpy.interp) within the rounding bound of
  a short positive-weight sum, so their separable summation order is one
  evaluation of the defined operator;
- the V-cycle equals a dense NumPy restatement of Alg. 2 whose transfer
  operators are built independently with numpy.interp and Kronecker products;
- on a grid that is already the coarsest level the V-cycle is the exact
  inverse, and MGCG converges in one iteration;
- the V-cycle is a symmetric positive definite operator (so PCG applies);
- MGCG converges to the dense solution, in a number of iterations that grows
  only slowly as the grid is refined (the multigrid property).
"""
import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W


def interp_matrix(nf, nc):
    """1D linear interpolation from coarse nodes I/(nc+1) to fine nodes i/(nf+1),
    zero at both ends, built column by column with numpy.interp."""
    xf = np.arange(1, nf + 1) / (nf + 1)
    Xc = np.arange(0, nc + 2) / (nc + 1)
    P = np.zeros((nf, nc))
    for I in range(1, nc + 1):
        e = np.zeros(nc + 2)
        e[I] = 1.0
        P[:, I - 1] = np.interp(xf, Xc, e)
    return P


def dense_vcycle(spec, mu, b, nu, omega):
    O = oracle.Problem(spec)
    ns = O.mg_levels()
    A = [oracle.Problem(W.scaled(spec, n)).dense(mu) for n in ns]
    Ps = []
    for l in range(len(ns) - 1):
        p1 = interp_matrix(ns[l], ns[l + 1])
        Ps.append(np.kron(np.kron(p1, p1), p1))     # x fastest: z (x) y (x) x

    def cyc(l, b):
        if l == len(ns) - 1:
            return np.linalg.solve(A[l], b)
        d = np.diag(A[l])
        e = np.zeros_like(b)
        for _ in range(nu):
            e = e + omega * (b - A[l] @ e) / d
        r = b - A[l] @ e
        rc = (ns[l + 1] + 1) / (ns[l] + 1) * (Ps[l].T @ r)
        e = e + Ps[l] @ cyc(l + 1, rc)
        for _ in range(nu):
            e = e + omega * (b - A[l] @ e) / d
        return e

    return cyc(0, b)


def test_levels():
    lv = lambda n: oracle.Problem(W.Problem(n, W.KIND_OCTANTS)).mg_levels()
    assert lv(128) == [128, 63, 31, 15, 7, 3]
    assert lv(16) == [16, 7, 3]
    assert lv(96) == [96, 47, 23, 11, 5, 2]
    assert lv(3) == [3]
    assert lv(4) == [4, 1]


def test_interp_matrix_is_linear_interpolation():
    # the independent transfer reproduces linear functions away from the ends
    P = interp_matrix(16, 7)
    Xc = np.arange(1, 8) / 8
    xf = np.arange(1, 17) / 17
    g = 0.3 + 2.0 * Xc
    inner = (xf >= Xc[0]) & (xf <= Xc[-1])
    np.testing.assert_allclose((P @ g)[inner], (0.3 + 2.0 * xf)[inner], rtol=1e-14)


@pytest.mark.parametrize("n,level", [(8, 0), (16, 0), (16, 1), (20, 0), (33, 0), (33, 1)])
def test_transfers_per_entry_match_kronecker(n, level):
    O = oracle.Problem(W.Problem(n, W.KIND_OCTANTS))
    ns = O.mg_levels()
    nf, nc = ns[level], ns[level + 1]
    p1 = interp_matrix(nf, nc)
    P = np.kron(np.kron(p1, p1), p1)
    scale = (nc + 1) / (nf + 1)
    rng = np.random.default_rng(n + level)
    eps = np.finfo(float).eps
    r = rng.standard_normal(nf ** 3) * np.exp(rng.uniform(-3, 3, nf ** 3))
    rc = O.mg_transfer(level, r, restrict=True)
    ref = scale * (P.T @ r)
    bound = 32 * eps * scale * (np.abs(P.T) @ np.abs(r)) + 1e-300
    assert (np.abs(rc - ref) <= bound).all(), np.max(np.abs(rc - ref) / bound)
    e = rng.standard_normal(nc ** 3)
    ef = O.mg_transfer(level, e, restrict=False)
    ref = P @ e
    bound = 32 * eps * (np.abs(P) @ np.abs(e)) + 1e-300
    assert (np.abs(ef - ref) <= bound).all(), np.max(np.abs(ef - ref) / bound)
    # and the pair is adjoint up to the scale: <R r, e> = scale <r, P e>
    assert abs(rc @ e - scale * (r @ ef)) <= 1e-12 * np.abs(rc) @ np.abs(e)


@pytest.mark.parametrize("spec", [W.Problem(8, W.KIND_OCTANTS), W.Problem(16, W.KIND_BLOCKS, W.BLOCKS3),
                                  W.Problem(10, W.KIND_OCTANTS_ANISO)], ids=["oct8", "blk16", "aniso10"])
@pytest.mark.parametrize("nu,omega", [(1, 6.0 / 7.0), (2, 0.8)])
def test_vcycle_matches_dense_restatement(spec, nu, omega):
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.05, 20.0, 1, 3)[0]
    b = np.random.default_rng(4).standard_normal(O.ndof)
    s = O.mg_apply(mu, b, nu, omega)
    ref = dense_vcycle(spec, mu, b, nu, omega)
    assert np.linalg.norm(s - ref) <= 1e-12 * np.linalg.norm(ref)


def test_coarsest_grid_is_exact():
    spec = W.Problem(3, W.KIND_OCTANTS)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 1, 5)[0]
    b = np.random.default_rng(1).standard_normal(O.ndof)
    np.testing.assert_allclose(O.mg_apply(mu, b), np.linalg.solve(O.dense(mu), b), rtol=1e-13, atol=1e-15)
    x, st = O.mgcg(mu, tol=1e-12)
    assert st["status"] == oracle.CONVERGED and st["iters"] == 1


def test_vcycle_is_spd():
    spec = W.Problem(8, W.KIND_OCTANTS)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 1, 6)[0]
    Bm = np.stack([O.mg_apply(mu, e) for e in np.eye(O.ndof)], axis=1)
    assert np.abs(Bm - Bm.T).max() <= 1e-12 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0
    # the preconditioned spectrum is clustered (multigrid), unlike Jacobi's
    A = O.dense(mu)
    ev = np.sort(np.linalg.eigvals(Bm @ A).real)
    evj = np.sort(np.linalg.eigvals(A / np.diag(A)[:, None]).real)
    assert ev[0] > 0 and ev[-1] / ev[0] < 0.2 * evj[-1] / evj[0]


def test_mgcg_solves_and_scales():
    its = []
    for n in (8, 16, 32):
        spec = W.Problem(n, W.KIND_OCTANTS)
        O = oracle.Problem(spec)
        mu = W.sample_mu(spec, 0.01, 100.0, 1, 7)[0]
        x, st = O.mgcg(mu, tol=1e-11)
        assert st["status"] == oracle.CONVERGED
        its.append(st["iters"])
        if n == 8:
            ref = np.linalg.solve(O.dense(mu), O.rhs(mu))
            assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
        xj, sj = O.cg(mu, tol=1e-11)
        if n >= 16:
            assert st["iters"] * 3 < sj["iters"]
    assert its[2] <= 1.5 * its[1] and its[1] <= 1.5 * its[0] + 2, its
