"""Pins for the oracle's finite-difference operator A_h(mu) and source f_h.

Model problem: -div(kappa(mu) grad u) = f on (0,1)^3 with zero Dirichlet data
(the paper's Sec. 4 model PDE, Eq. 1 for the discrete system), 7-point finite
differences on an n^3 interior grid, unscaled form
    (A u)_P = sum over the 6 faces of P of kappa_f (u_P - u_nb),  f_h = h^2 f.

Pins: hand-derived matrices and face values on tiny grids (including the
sub-domain tie rule and painter's order of overlapping blocks), exact
symmetry, diagonal dominance, positive definiteness, the affine split
A(mu) = sum_q theta_q A_q with each A_q positive semi-definite, and the
discrete sine eigenvector that gives a closed-form solution and the O(h^2)
error of the scheme.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W


def test_octants_n2_hand_derived():
    # n = 2: node (i,j,k) sits alone in octant o = (i-1) + 2(j-1) + 4(k-1).
    # Boundary faces carry mu_o; the interior face between two nodes lies on
    # the split plane x|y|z = 1/2, so it carries the mean (mu_o + mu_o')/2.
    rng = np.random.default_rng(3)
    mu = 10.0 ** rng.uniform(-1, 1, 8)
    P = oracle.Problem(W.Problem(2, W.KIND_OCTANTS))
    A = P.dense(mu)
    E = np.zeros((8, 8))
    for o in range(8):
        E[o, o] = 3 * mu[o]
        for bit in range(3):
            nb = o ^ (1 << bit)
            kf = (mu[o] + mu[nb]) / 2
            E[o, o] += kf
            E[o, nb] = -kf
    np.testing.assert_allclose(A, E, rtol=1e-15, atol=0)


def test_block_tie_rule_hand_derived():
    # n = 4 (h = 0.2), one block [0.1,0.4]^3 with kappa = mu inside, 1 outside.
    P = oracle.Problem(W.Problem(4, W.KIND_BLOCKS, ((1, 4, 1, 4, 1, 4),)))
    mu = 5.0
    kx, ky, kz = P.face_coeffs([1.0, mu])
    n = 4

    def KX(i, j, k):  # face between x-nodes i, i+1 at (j, k)
        return kx[((k - 1) * n + (j - 1)) * (n + 1) + i]

    def KY(i, j, k):
        return ky[((k - 1) * (n + 1) + j) * n + (i - 1)]

    def KZ(i, j, k):
        return kz[(k * n + (j - 1)) * n + (i - 1)]

    assert KX(1, 1, 1) == mu                     # x = 0.3 strictly inside
    assert KX(0, 1, 1) == (1 + mu) / 2           # x = 0.1 on the block face
    assert KX(1, 2, 1) == (mu + 1) / 2           # y = 0.4 on the block face
    assert KX(1, 2, 2) == (mu + 3) / 4           # y, z on faces: 1 of 4 corners inside
    assert KX(0, 2, 2) == (mu + 7) / 8           # x, y, z on faces: 1 of 8 corners inside
    assert KX(2, 1, 1) == 1.0                    # x = 0.5 outside
    assert KY(1, 0, 1) == (1 + mu) / 2
    assert KZ(1, 1, 4) == 1.0


def test_painters_order():
    # n = 19: the x-face at x = 0.325, y = z = 0.35 lies strictly inside both
    # [0.1,0.4]^3 and [0.3,0.7]^3; the last-listed block decides its value.
    n = 19
    i, j, k = 6, 7, 7
    for blocks, want in ((((1, 4, 1, 4, 1, 4), (3, 7, 3, 7, 3, 7)), 3.0),
                         (((3, 7, 3, 7, 3, 7), (1, 4, 1, 4, 1, 4)), 3.0)):
        P = oracle.Problem(W.Problem(n, W.KIND_BLOCKS, blocks))
        kx, _, _ = P.face_coeffs([1.0, 2.0, 3.0])
        assert kx[((k - 1) * n + (j - 1)) * (n + 1) + i] == want


@pytest.mark.parametrize("spec", [W.Problem(5, W.KIND_BLOCKS, W.BLOCKS3),
                                  W.Problem(6, W.KIND_BLOCKS, W.BLOCKS4),
                                  W.Problem(5, W.KIND_OCTANTS),
                                  W.Problem(4, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS)])
def test_symmetric_dominant_spd(spec):
    P = oracle.Problem(spec)
    rng = np.random.default_rng(11)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 5)
    for m in mu:
        A = P.dense(m)
        assert np.array_equal(A, A.T)                       # same face, same value
        off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
        assert np.all(np.diag(A) >= off * (1 - 1e-15))
        assert np.any(np.diag(A) > off * (1 + 1e-3))         # boundary rows strictly
        np.linalg.cholesky(A)                                 # positive definite
        x, y = rng.standard_normal(P.ndof), rng.standard_normal(P.ndof)
        a, b = x @ P.apply(m, y), y @ P.apply(m, x)
        assert abs(a - b) <= 1e-14 * np.abs(A).max() * np.abs(x).sum() * np.abs(y).max()


@pytest.mark.parametrize("spec", [W.Problem(5, W.KIND_BLOCKS, W.BLOCKS4),
                                  W.Problem(4, W.KIND_OCTANTS),
                                  W.Problem(4, W.KIND_OCTANTS_ANISO)])
def test_affine_split(spec):
    P = oracle.Problem(spec)
    rng = np.random.default_rng(2)
    mu = W.sample_mu(spec, 0.1, 10.0, 1, 9)[0]
    th = P.theta(mu)
    x = rng.standard_normal(P.ndof)
    parts = []
    for q in range(P.Q):
        e = np.zeros(P.Q)
        e[q] = 1.0
        Aq = np.stack([P.apply_theta(e, col) for col in np.eye(P.ndof)], axis=1)
        assert np.linalg.eigvalsh(Aq).min() >= -1e-12        # each A_q is PSD
        parts.append(th[q] * (Aq @ x))
    lhs = P.apply(mu, x)
    np.testing.assert_allclose(lhs, np.sum(parts, axis=0), rtol=1e-12,
                               atol=1e-12 * np.abs(lhs).max())


def sine_mode(n):
    h = 1.0 / (n + 1)
    g = np.sin(np.pi * h * np.arange(1, n + 1))
    return np.einsum("k,j,i->kji", g, g, g).reshape(-1), h


@pytest.mark.parametrize("n", [3, 8, 17])
def test_sine_eigenvector(n):
    # w_P = sin(pi x) sin(pi y) sin(pi z): A w = 4 sin^2(pi h/2)(kx+ky+kz) w
    w, h = sine_mode(n)
    lam1 = 4 * math.sin(math.pi * h / 2) ** 2
    Piso = oracle.Problem(W.Problem(n, W.KIND_OCTANTS))
    np.testing.assert_allclose(Piso.apply(np.full(8, 1.0), w), 3 * lam1 * w, rtol=1e-13,
                               atol=1e-14)
    Pan = oracle.Problem(W.Problem(n, W.KIND_OCTANTS_ANISO))
    kap = np.tile([0.5, 2.0, 7.0], 8)
    np.testing.assert_allclose(Pan.apply(kap, w), (0.5 + 2.0 + 7.0) * lam1 * w, rtol=1e-13,
                               atol=1e-13)


@pytest.mark.parametrize("n,err", [(16, 2.8508e-3), (32, 7.5559e-4)])
def test_manufactured_solution_and_order(n, err):
    # f = 3 pi^2 sin sin sin has u = sin sin sin.  Discretely, u_h is the sine
    # mode times pi^2 h^2 / (4 sin^2(pi h / 2)), so the nodal error is
    # pi^2 h^2 / (4 sin^2(pi h/2)) - 1 ~ pi^2 h^2 / 12: second order.
    w, h = sine_mode(n)
    P = oracle.Problem(W.Problem(n, W.KIND_OCTANTS))
    f = h * h * 3 * math.pi ** 2 * w
    u, st = P.cg(np.ones(8), f=f, prec=oracle.PREC_NONE, tol=1e-12, maxit=5)
    assert st["status"] == oracle.CONVERGED and st["iters"] == 1
    scale = math.pi ** 2 * h * h / (4 * math.sin(math.pi * h / 2) ** 2)
    np.testing.assert_allclose(u, scale * w, rtol=1e-13, atol=1e-15)
    rel = np.abs(u - w).max() / np.abs(w).max()
    assert abs(rel - err) < 1e-7
    assert abs(rel / (math.pi ** 2 * h * h / 12) - 1) < 0.01


def test_rhs_and_theta():
    spec = W.Problem(3, W.KIND_BLOCKS, W.BLOCKS3)
    P = oracle.Problem(spec)
    f = P.rhs([1.0, 2.0, 3.0])
    assert np.all(f == (1.0 / 4) * (1.0 / 4))
    np.testing.assert_array_equal(P.theta([2.0, 3.0, 4.0]), [1.0, 2.0, 3.0, 4.0])
    g = oracle.Problem(W.Problem(3, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02))
    mu = np.concatenate([np.ones(24), [0.5, 0.5, 0.5]])
    fg = g.rhs(mu)
    # centre node sits at the Gaussian's centre: f = h^2 exp(0)
    assert fg[13] == (1.0 / 4) ** 2
    assert fg[0] == pytest.approx((1 / 16) * math.exp(-3 * 0.25 ** 2 / 0.02), rel=1e-15)
