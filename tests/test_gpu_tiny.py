"""GPU parity on the smallest grids the library accepts, through the C ABI.

n = 1 is a single unknown, whose stencil has no interior neighbour. n = 2 is a
quad that is only half used. n = 4 and 5 give whole and partial quads on a
grid with one row of tiles. Their V-cycles have a finest level that is already
the coarsest (n <= 3: an exact solve), or a single coarser level. The FP64
results are the oracle's bit for bit. The FP32 inner / FP64 outer refinement
matches its FP64 solution to 1e-8."""
import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    from paper_2311_13862_amd import rbws
    assert torch.cuda.is_available()
    return rbws


TINY = [W.Problem(1, W.KIND_OCTANTS), W.Problem(2, W.KIND_OCTANTS), W.Problem(1, W.KIND_BLOCKS, W.BLOCKS4),
        W.Problem(2, W.KIND_BLOCKS, W.BLOCKS3), W.Problem(2, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02),
        W.Problem(4, W.KIND_OCTANTS), W.Problem(5, W.KIND_OCTANTS_ANISO)]
IDS = [f"k{s.kind}n{s.n}" + ("g" if s.f_kind == W.F_GAUSS else "") for s in TINY]


def solve(rb, spec, mu, opts):
    P = rb.Problem(spec)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mu))]
    st = rb.solve([P], mu, opts, u_out=u)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in u], st


@pytest.mark.parametrize("spec", TINY, ids=IDS)
def test_tiny_spmv_fp64_bitwise(rb, spec):
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 7)
    x = np.random.default_rng(spec.n).standard_normal((3, P.ndof))
    y = torch.empty((3, P.ndof), dtype=torch.float64, device="cuda")
    P.spmv(mu, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    for b in range(3):
        assert np.array_equal(got[b], O.apply(mu[b], x[b])), b


@pytest.mark.parametrize("spec", TINY, ids=IDS)
@pytest.mark.parametrize("prec", [0, 1])
def test_tiny_cg_bitwise(rb, spec, prec):
    """Alg. 1 with P = I and P = Jacobi: iteration counts, residuals and
    solutions of the oracle."""
    mu = W.sample_mu(spec, 0.01, 100.0, 4, 11)
    xg, sg = solve(rb, spec, mu, rb.default_opts(tol=1e-11, precond=prec))
    xo, so = oracle.Problem(spec).cg_batch(mu, prec=prec, tol=1e-11)
    for b in range(len(mu)):
        assert sg[b]["status"] == so[b]["status"] == 0
        assert sg[b]["iters"] == so[b]["iters"], (b, sg[b]["iters"], so[b]["iters"])
        assert sg[b]["final_rr"] == so[b]["final_rr"] and sg[b]["ff"] == so[b]["ff"]
        assert np.array_equal(xg[b], xo[b]), b


@pytest.mark.parametrize("spec", TINY, ids=IDS)
def test_tiny_mgcg_and_vcycle_bitwise(rb, spec):
    """Alg. 1 preconditioned by the V-cycle of Alg. 2 (FP64), and one V-cycle
    through rbws_mg_apply, against the oracle."""
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 4, 13)
    opts = rb.default_opts(tol=1e-11, precond=rb.PREC_MG, mg_nu=1, mg_omega=6.0 / 7.0)
    xg, sg = solve(rb, spec, mu, opts)
    xo, so = O.mgcg_batch(mu, nu=1, omega=6.0 / 7.0, tol=1e-11)
    for b in range(len(mu)):
        assert sg[b]["status"] == so[b]["status"] == 0
        assert sg[b]["iters"] == so[b]["iters"], (b, sg[b]["iters"], so[b]["iters"])
        assert np.array_equal(xg[b], xo[b]), b
    P = rb.Problem(spec)
    rhs = np.random.default_rng(3 + spec.n).standard_normal((len(mu), O.ndof))
    s = torch.empty((len(mu), O.ndof), dtype=torch.float64, device="cuda")
    P.mg_apply(mu, torch.from_numpy(rhs).cuda(), s, nu=1, omega=6.0 / 7.0)
    torch.cuda.synchronize()
    sv = s.cpu().numpy()
    for b in range(len(mu)):
        assert np.array_equal(sv[b], O.mg_apply(mu[b], rhs[b], 1, 6.0 / 7.0)), b


@pytest.mark.parametrize("spec", TINY, ids=IDS)
@pytest.mark.parametrize("precond", [1, 2])
def test_tiny_refinement(rb, spec, precond):
    """FP32 inner (Jacobi or V-cycle PCG) / FP64 outer refinement to 1e-10:
    converged, and within 1e-8 of the oracle's FP64 solution."""
    mu = W.sample_mu(spec, 0.01, 100.0, 4, 17)
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=precond, ir_mode=rb.IR_RELIABLE,
                           eta_inner=0.05)
    xg, sg = solve(rb, spec, mu, opts)
    ref, _ = oracle.Problem(spec).cg_batch(mu, tol=1e-13, maxit=20000)
    for b in range(len(mu)):
        assert sg[b]["status"] == rb.SOLVE_CONVERGED, (b, sg[b]["status"])
        assert sg[b]["final_rr"] <= 1e-20 * sg[b]["ff"]
        assert np.linalg.norm(xg[b] - ref[b]) <= 1e-8 * np.linalg.norm(ref[b]), b
