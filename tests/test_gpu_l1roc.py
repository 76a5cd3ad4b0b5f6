"""GPU L1ROC (Sec. 3.1, Alg. 4) against the oracle: the greedy (selections,
DEIM points, basis, T, indicators), the collocation least-squares
coefficients and the warm-started solve, bit for bit for f = 1 (up to N = 60),
to stated tolerances for the Gaussian source; error paths."""
import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_13862_amd import rbws
    return rbws


def basis_v(rb, basis):
    V = np.empty((basis.N, basis.problem.ndof))
    rb._check(rb._L.rbws_basis_get(basis.handle, rb._dp(V), None, None))
    return V


CASES = [("blocks16", W.Problem(16, W.KIND_BLOCKS, W.BLOCKS3), 0.1, 10.0, 256, 10),
         ("octants12", W.Problem(12, W.KIND_OCTANTS), 0.01, 100.0, 64, 8)]


@pytest.mark.parametrize("name,spec,lo,hi,nt,N", CASES, ids=[c[0] for c in CASES])
def test_l1roc_greedy_bitwise(rb, name, spec, lo, hi, nt, N):
    mut = W.sample_mu(spec, lo, hi, nt, W.SEED_TRAIN)
    P = rb.Problem(spec)
    gb = rb.Basis.build(P, mut, N, 1e-13, method="l1roc")
    ob = oracle.l1roc_greedy(oracle.Problem(spec), mut, N, 1e-13)
    info = gb.l1roc_info()
    assert list(gb.selected) == list(ob.selected)
    assert list(info["xs"]) == list(ob.xs) and list(info["xr"]) == list(ob.xr)
    assert list(info["pts"]) == list(ob.pts)
    assert np.array_equal(basis_v(rb, gb), ob.W)
    assert np.array_equal(info["T"], ob.T)
    assert np.array_equal(gb.hist, ob.hist)


@pytest.fixture(scope="module")
def l1pair(rb):
    wl = W.blocks3_16()
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    P = rb.Problem(wl.problem)
    gb = rb.Basis.build(P, mut, 12, wl.snap_tol, method="l1roc")
    ob = oracle.l1roc_greedy(oracle.Problem(wl.problem), mut, 12, wl.snap_tol)
    return wl, P, gb, ob


def test_l1roc_coeffs_bitwise(rb, l1pair):
    wl, P, gb, ob = l1pair
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 8, W.SEED_TEST)
    cg = gb.coeffs(mus)
    for b, mu in enumerate(mus):
        assert np.array_equal(cg[b], ob.coeffs(mu)), b


def test_l1roc_warm_start_bitwise(rb, l1pair):
    """FP64 PCG from the L1ROC start: iterations, residuals and solutions equal
    to the oracle's Alg. 5 with the same start, and fewer iterations than from
    zero."""
    wl, P, gb, ob = l1pair
    O = oracle.Problem(wl.problem)
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 6, W.SEED_TEST)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
    st = rb.solve([P], mus, rb.default_opts(tol=wl.tol, init=rb.INIT_RB), bases=[gb], u_out=u)
    zs = rb.solve([P], mus, rb.default_opts(tol=wl.tol))
    for b, mu in enumerate(mus):
        xo, so = O.cg(mu, u0=ob.lift(ob.coeffs(mu)), tol=wl.tol)
        assert st[b]["iters"] == so["iters"] and st[b]["final_rr"] == so["final_rr"]
        assert np.array_equal(u[b].cpu().numpy(), xo)
        assert st[b]["iters"] < zs[b]["iters"]


def test_l1roc_start_in_refinement(rb):
    """FP32 V-cycle CG in FP64 refinement from the L1ROC start at 40^3: all
    solves converge and match the oracle's FP64 solution to 1e-8."""
    spec = W.Problem(40, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mut = W.sample_mu(spec, 0.01, 100.0, 48, W.SEED_TRAIN)
    gb = rb.Basis.build(P, mut, 8, 1e-12, method="l1roc")
    mus = W.sample_mu(spec, 0.01, 100.0, 4, W.SEED_TEST)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=rb.PREC_MG, init=rb.INIT_RB, eta_inner=0.05,
                           mg_omega=0.9)
    st = rb.solve([P], mus, opts, bases=[gb], u_out=u)
    ref, _ = O.mgcg_batch(mus, tol=1e-12)
    for b in range(len(mus)):
        assert st[b]["status"] == rb.SOLVE_CONVERGED
        ub = u[b].cpu().numpy()
        assert np.linalg.norm(ub - ref[b]) <= 1e-8 * np.linalg.norm(ref[b])


@pytest.fixture(scope="module")
def l1gauss(rb):
    """Anisotropic octants with the Gaussian source at 12^3 (27 parameters): the
    source enters the collocation problem through its M point values."""
    spec = W.Problem(12, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02)
    # (with a small training set the L1 indicator's maximiser is the first
    # parameter again and the greedy stops at one vector: f is concentrated
    # near x0, so few parameters have a large coefficient at the first point)
    mut = W.sample_mu(spec, 0.1, 10.0, 1024, W.SEED_TRAIN)
    P = rb.Problem(spec)
    gb = rb.Basis.build(P, mut, 10, 1e-12, method="l1roc")
    ob = oracle.l1roc_greedy(oracle.Problem(spec), mut, 10, 1e-12)
    return spec, mut, P, gb, ob


def test_l1roc_gaussian_greedy(rb, l1gauss):
    """Each side evaluates the source with its own exp, which may differ in the
    last bit, so the greedy is compared to tolerances where a choice is not a
    near-tie: the same parameters, DEIM points, W and T to 1e-9, indicators to
    1e-7."""
    spec, mut, P, gb, ob = l1gauss
    assert gb.N == ob.N
    for k in range(gb.N - 1):
        row = np.sort(ob.hist[k])[::-1]
        assert row[0] > row[1] * (1 + 1e-6), k
    info = gb.l1roc_info()
    assert list(gb.selected) == list(ob.selected)
    assert list(info["xs"]) == list(ob.xs) and list(info["xr"]) == list(ob.xr)
    assert list(info["pts"]) == list(ob.pts)
    assert np.abs(basis_v(rb, gb) - ob.W).max() <= 1e-9 * np.abs(ob.W).max()
    np.testing.assert_allclose(info["T"], ob.T, rtol=1e-9, atol=1e-9 * np.abs(ob.T).max())
    np.testing.assert_allclose(gb.hist, ob.hist, rtol=1e-7)


def test_l1roc_gaussian_online_and_refinement(rb, l1gauss):
    """Collocation coefficients at held-out parameters to 1e-9 of the oracle's,
    and FP32 V-cycle CG in FP64 refinement from the L1ROC start matching the
    oracle's FP64 MGCG to 1e-8."""
    spec, mut, P, gb, ob = l1gauss
    mus = W.sample_mu(spec, 0.1, 10.0, 6, W.SEED_TEST)
    c = gb.coeffs(mus)
    for b, mu in enumerate(mus):
        co = ob.coeffs(mu)
        assert np.linalg.norm(c[b] - co) <= 1e-9 * np.linalg.norm(co), b
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=rb.PREC_MG, init=rb.INIT_RB, eta_inner=0.05,
                           mg_omega=0.9)
    st = rb.solve([P], mus, opts, bases=[gb], u_out=u)
    O = oracle.Problem(spec)
    for b, mu in enumerate(mus):
        assert st[b]["status"] == rb.SOLVE_CONVERGED
        ref, so = O.mgcg(mu, tol=1e-12)
        ub = u[b].cpu().numpy()
        assert np.linalg.norm(ub - ref) <= 1e-8 * np.linalg.norm(ref), b


def test_l1roc_sixty_vectors(rb):
    """N = 60 (M up to 119 collocation rows in LDS) on a 16^3 block problem,
    bit for bit against the oracle, as far as the greedy runs."""
    spec = W.Problem(16, W.KIND_BLOCKS, W.BLOCKS4)
    mut = W.sample_mu(spec, 0.1, 10.0, 256, W.SEED_TRAIN)
    P = rb.Problem(spec)
    gb = rb.Basis.build(P, mut, 60, 1e-13, method="l1roc")
    ob = oracle.l1roc_greedy(oracle.Problem(spec), mut, 60, 1e-13)
    print("L1ROC greedy reached", gb.N, "points", len(gb.l1roc_info()["pts"]))
    assert gb.N == ob.N and gb.N > 40
    assert list(gb.selected) == list(ob.selected)
    assert np.array_equal(basis_v(rb, gb), ob.W)
    assert np.array_equal(gb.hist, ob.hist)
    mus = W.sample_mu(spec, 0.1, 10.0, 4, W.SEED_TEST)
    c = gb.coeffs(mus)
    for b, mu in enumerate(mus):
        assert np.array_equal(c[b], ob.coeffs(mu)), b


def test_l1roc_errors(rb):
    spec = W.Problem(8, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mut = W.sample_mu(spec, 0.01, 100.0, 64, 3)
    with pytest.raises(rb.RbwsError):
        rb.Basis.build(P, mut, 61, 1e-12, method="l1roc")  # N above 60
    gb = rb.Basis.build(P, mut, 4, 1e-12, method="l1roc")
    with pytest.raises(rb.RbwsError):
        gb.save("/dev/null")
    galerkin = rb.Basis.build(P, mut, 4, 1e-12)
    with pytest.raises(rb.RbwsError):
        galerkin.l1roc_info()
