"""Pins of the oracle's L1ROC (Sec. 3.1, Alg. 4): a dense NumPy restatement on
a tiny grid, the DEIM structure, the least-squares solve, exact reproduction
of the chosen snapshots, and the warm start's saving."""
import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W


def pick(values, expected):
    """argmax, except that an expected index whose value is within 1e-9 of the
    maximum is taken instead: exact ties (from the problems' symmetries) are
    broken by rounding, and any near-maximal choice is a correct one."""
    v = np.asarray(values)
    if expected is not None and v[expected] >= v.max() * (1.0 - 1e-9):
        return int(expected)
    return int(np.argmax(v))


def l1roc_dense(O, mut, N, follow=None):
    """Alg. 4 written out with dense NumPy algebra: snapshots by dense solves,
    DEIM by a dense triangular solve and argmax, the collocation problem by
    numpy.linalg.lstsq, and the L1 indicator from a least-squares fit of the
    snapshots themselves (no use of the oracle's T).  `follow` (an oracle
    basis) resolves near-ties in favour of the oracle's choice (see pick)."""
    A = lambda mu: O.dense(mu)
    f = lambda mu: O.rhs(mu)
    exp = lambda seq, i: int(seq[i]) if follow is not None and i < len(seq) else None

    def deim(B, pts, x, expected):
        nb = len(pts)
        r = x.copy()
        if nb:
            M = np.array([[B[j][pts[i]] for j in range(nb)] for i in range(nb)])
            c = np.linalg.solve(M, x[pts])
            r = x - np.array(B).T @ c
        r[pts] = 0.0
        k = pick(np.abs(r), expected)
        return k, r / r[k]

    def lsq(Wl, P, mu):
        M = (A(mu) @ np.array(Wl).T)[P]
        return np.linalg.lstsq(M, f(mu)[P], rcond=None)[0]

    u = np.linalg.solve(A(mut[0]), f(mut[0]))
    k, w = deim([], [], u, exp(follow.xs, 0) if follow is not None else None)
    Wl, xs, xr, R, sel, snaps, hist = [w], [k], [], [], [0], [u], []
    while True:
        P = sorted(set(xs) | set(xr))
        U = np.array(snaps).T
        ind = []
        for mu in mut:
            cu = np.linalg.lstsq(U, np.array(Wl).T @ lsq(Wl, P, mu), rcond=None)[0]
            ind.append(np.abs(cu).sum())
        hist.append(ind)
        if len(Wl) == N:
            break
        best = pick(ind, exp(follow.selected, len(sel)) if follow is not None else None)
        if best in sel:
            break
        mu = mut[best]
        r = f(mu) - A(mu) @ (np.array(Wl).T @ lsq(Wl, P, mu))
        u = np.linalg.solve(A(mu), f(mu))
        k, w = deim(Wl, xs, u, exp(follow.xs, len(xs)) if follow is not None else None)
        Wl.append(w)
        xs.append(k)
        snaps.append(u)
        kr, wr = deim(R, xr, r, exp(follow.xr, len(xr)) if follow is not None else None)
        R.append(wr)
        xr.append(kr)
        sel.append(best)
    return np.array(Wl), xs, xr, sel, np.array(hist)


@pytest.mark.parametrize("kind", [W.KIND_BLOCKS, W.KIND_OCTANTS, W.KIND_OCTANTS_ANISO])
def test_l1roc_matches_dense_restatement(kind):
    """Blocks and octants (f = 1), and anisotropic octants with the Gaussian
    source, whose collocation right-hand side is f(mu) at the points."""
    if kind == W.KIND_BLOCKS:
        spec, lo, hi = W.Problem(5, kind, W.BLOCKS3), 0.1, 10.0
    elif kind == W.KIND_OCTANTS:
        spec, lo, hi = W.Problem(5, kind), 0.01, 100.0
    else:
        spec, lo, hi = W.Problem(5, kind, (), W.F_GAUSS, 0.02), 0.1, 10.0
    O = oracle.Problem(spec)
    mut = W.sample_mu(spec, lo, hi, 16, 21 + kind)
    B = oracle.l1roc_greedy(O, mut, 5, 1e-14)
    Wd, xs, xr, sel, hist = l1roc_dense(O, mut, 5, follow=B)
    assert list(B.selected) == sel
    assert list(B.xs) == xs and list(B.xr) == xr
    assert list(B.pts) == sorted(set(xs) | set(xr))
    np.testing.assert_allclose(B.W, Wd, rtol=0, atol=1e-9 * np.abs(Wd).max())
    np.testing.assert_allclose(B.hist, hist, rtol=1e-7)


@pytest.fixture(scope="module")
def l1_16():
    wl = W.blocks3_16()
    O = oracle.Problem(wl.problem)
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    return wl, O, mut, oracle.l1roc_greedy(O, mut, 10, wl.snap_tol)


def test_deim_structure_and_snapshot_basis(l1_16):
    """W_j[x_j] = 1 and W_j[x_i] = 0 for i < j at the snapshot points; T is
    upper triangular and W = U T with U the snapshots solved again here."""
    wl, O, mut, B = l1_16
    for j in range(B.N):
        assert B.W[j][B.xs[j]] == 1.0
        assert all(B.W[j][B.xs[i]] == 0.0 for i in range(j))
    assert np.array_equal(np.triu(B.T), B.T)
    U = np.array([O.cg(mut[s], tol=1e-13)[0] for s in B.selected]).T
    np.testing.assert_allclose(U @ B.T, B.W.T, rtol=0, atol=1e-9 * np.abs(B.W).max())
    assert len(B.pts) <= 2 * B.N - 1 and np.all(np.diff(B.pts) > 0)


def test_collocation_least_squares(l1_16):
    """The oracle's Householder QR against numpy.linalg.lstsq on the same
    rows (A(mu) W)[X], f[X], the rows formed here with a dense operator."""
    wl, O, mut, B = l1_16
    for mu in W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 4, 77):
        M = (O.dense(mu) @ B.W.T)[B.pts]
        ref = np.linalg.lstsq(M, O.rhs(mu)[B.pts], rcond=None)[0]
        np.testing.assert_allclose(B.coeffs(mu), ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_selected_snapshots_reproduced(l1_16):
    """A chosen parameter's snapshot lies in span(W): the collocation solve
    reproduces it up to the snapshot tolerance."""
    wl, O, mut, B = l1_16
    for s in B.selected:
        u = O.cg(mut[s], tol=1e-13)[0]
        err = np.linalg.norm(B.lift(B.coeffs(mut[s])) - u) / np.linalg.norm(u)
        assert err < 1e-9, (s, err)


def test_l1roc_warm_start_saves_iterations(l1_16):
    """The L1ROC start needs fewer PCG iterations than the zero start (Sec. 4)."""
    wl, O, mut, B = l1_16
    for mu in W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 6, W.SEED_TEST):
        _, sz = O.cg(mu, tol=wl.tol)
        _, sw = O.cg(mu, u0=B.lift(B.coeffs(mu)), tol=wl.tol)
        assert sw["status"] == oracle.CONVERGED and sw["iters"] < sz["iters"], (sw["iters"], sz["iters"])


@pytest.mark.parametrize("seed", range(4))
def test_collocation_qr_random(seed):
    """The oracle's Householder QR on arbitrary bases and point sets (not just
    the greedy's DEIM-structured ones) against numpy.linalg.lstsq."""
    rng = np.random.default_rng(seed)
    spec = W.Problem(6, W.KIND_OCTANTS)
    O = oracle.Problem(spec)
    N = 3 + seed
    M = N + 1 + 2 * seed
    Wr = rng.standard_normal((N, O.ndof))
    pts = np.sort(rng.choice(O.ndof, size=M, replace=False)).astype(np.int64)
    B = oracle.L1rocBasis(O, Wr, np.eye(N), pts, pts[:N], pts[N:], np.arange(N), None)
    mu = W.sample_mu(spec, 0.01, 100.0, 1, 50 + seed)[0]
    ref = np.linalg.lstsq((O.dense(mu) @ Wr.T)[pts], O.rhs(mu)[pts], rcond=None)[0]
    np.testing.assert_allclose(B.coeffs(mu), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
