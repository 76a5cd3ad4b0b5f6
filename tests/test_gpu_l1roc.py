"""GPU L1ROC (Sec. 3.1, Alg. 4) against the oracle: the greedy (selections,
DEIM points, basis, T, indicators), the collocation least-squares
coefficients and the warm-started solve, bit for bit; error paths."""
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


def test_l1roc_errors(rb):
    spec = W.Problem(8, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mut = W.sample_mu(spec, 0.01, 100.0, 64, 3)
    with pytest.raises(rb.RbwsError):
        rb.Basis.build(P, mut, 41, 1e-12, method="l1roc")  # N above 40
    g = rb.Problem(W.Problem(8, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02))
    with pytest.raises(rb.RbwsError):
        rb.Basis.build(g, W.sample_mu(g.spec, 0.1, 10.0, 8, 1), 3, 1e-12, method="l1roc")  # f not constant
    gb = rb.Basis.build(P, mut, 4, 1e-12, method="l1roc")
    with pytest.raises(rb.RbwsError):
        gb.save("/dev/null")
    galerkin = rb.Basis.build(P, mut, 4, 1e-12)
    with pytest.raises(rb.RbwsError):
        galerkin.l1roc_info()
