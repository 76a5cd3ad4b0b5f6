"""GPU parity of MGCG (Alg. 1 preconditioned by the V-cycle of Alg. 2)
against the oracle, through the C ABI.

Every step of the V-cycle has a fixed evaluation order on both sides and the
inner products of PCG are correctly rounded, so the FP64 trajectories agree
bit for bit: iteration counts, residuals and solutions."""
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


def gpu_mgcg(rb, probs, mu, tol, nu=1, omega=6.0 / 7.0, problem_of=None, init=0, bases=None, flags=0):
    u = [torch.empty(probs[q].ndof, dtype=torch.float64, device="cuda")
         for q in (problem_of if problem_of is not None else [0] * len(mu))]
    opts = rb.default_opts(tol=tol, precond=rb.PREC_MG, mg_nu=nu, mg_omega=omega, init=init, flags=flags)
    st = rb.solve(probs, mu, opts, problem_of=problem_of, bases=bases, u_out=u)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in u], st


CASES = [W.Problem(16, W.KIND_BLOCKS, W.BLOCKS3), W.Problem(20, W.KIND_OCTANTS),
         W.Problem(12, W.KIND_OCTANTS_ANISO), W.Problem(3, W.KIND_OCTANTS), W.Problem(33, W.KIND_BLOCKS, W.BLOCKS4)]


@pytest.mark.parametrize("spec", CASES, ids=lambda s: f"k{s.kind}n{s.n}")
@pytest.mark.parametrize("nu,omega", [(1, 6.0 / 7.0), (2, 0.8)])
def test_mgcg_parity(rb, spec, nu, omega):
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 5, 40 + spec.n)
    xg, sg = gpu_mgcg(rb, [P], mu, 1e-11, nu, omega)
    xo, so = O.mgcg_batch(mu, nu=nu, omega=omega, tol=1e-11)
    for b in range(len(mu)):
        assert sg[b]["status"] == so[b]["status"] == 0
        assert sg[b]["iters"] == so[b]["iters"], (b, sg[b]["iters"], so[b]["iters"])
        assert sg[b]["extra_spmv"] == so[b]["extra_spmv"]
        assert sg[b]["final_rr"] == so[b]["final_rr"] and sg[b]["init_rr"] == so[b]["init_rr"]
        assert np.array_equal(xg[b], xo[b])
    if spec.n >= 16:
        xj, sj = O.cg_batch(mu[:1], tol=1e-11)
        assert sg[0]["iters"] * 2 < sj[0]["iters"]


@pytest.mark.parametrize("spec", CASES, ids=lambda s: f"k{s.kind}n{s.n}")
@pytest.mark.parametrize("nu,omega", [(1, 6.0 / 7.0), (2, 0.8)])
def test_vcycle_operator_fp64(rb, spec, nu, omega):
    """rbws_mg_apply in FP64 is the oracle's V-cycle bit for bit."""
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 80 + spec.n)
    rhs = np.random.default_rng(spec.n).standard_normal((3, O.ndof))
    r = torch.tensor(rhs, device="cuda")
    s = torch.empty_like(r)
    P.mg_apply(mu, r, s, nu=nu, omega=omega)
    sg = s.cpu().numpy()
    for b in range(len(mu)):
        assert np.array_equal(sg[b], O.mg_apply(mu[b], rhs[b], nu, omega)), b


@pytest.mark.parametrize("spec", [W.Problem(64, W.KIND_OCTANTS), W.Problem(33, W.KIND_BLOCKS, W.BLOCKS4),
                                  W.Problem(20, W.KIND_OCTANTS_ANISO), W.Problem(128, W.KIND_OCTANTS),
                                  W.Problem(96, W.KIND_OCTANTS_ANISO), W.Problem(70, W.KIND_OCTANTS)],
                         ids=["oct64", "blk33", "aniso20", "oct128", "aniso96", "oct70"])
def test_vcycle_operator_fp32(rb, spec):
    """The FP32 V-cycle (float coefficients and vectors, reciprocal-diagonal
    Jacobi on the fused levels) against the oracle's FP64 one: relative 2-norm
    error within 2e-5, about 100 float roundings of accumulated error; a wrong
    weight, index or sign gives errors of order 1e-2 or more."""
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 4, 90 + spec.n)
    rhs = np.random.default_rng(spec.n + 1).standard_normal((4, O.ndof))
    r = torch.tensor(rhs, device="cuda", dtype=torch.float32)
    s = torch.empty_like(r)
    P.mg_apply(mu, r, s, precision=rb.FP32_IR)
    sg = s.double().cpu().numpy()
    for b in range(len(mu)):
        ref = O.mg_apply(mu[b], r[b].double().cpu().numpy(), 1, 6.0 / 7.0)
        err = np.linalg.norm(sg[b] - ref) / np.linalg.norm(ref)
        assert err <= 2e-5, (b, err)


@pytest.mark.parametrize("n", [20, 33, 64, 70, 72, 128, 129])
def test_vcycle_fp32_fused_interpolation_same_bits(rb, n):
    """Where a level's tiles span whole rows, the FP32 post-smoothing forms the
    z/y interpolation of the coarse correction itself (RBWS_TUNE_MG_PZ = 1)
    with the same operations as the separate pass (0): the V-cycle gives the
    same bits either way.  The sizes cover 32 x 32 (n <= 32), 64 x 16 and
    128 x 8 whole-row tiles, scalar row ends (70), and n = 129, whose finest
    level has 32 x 32 tiles that do not span the row."""
    spec = W.Problem(n, W.KIND_OCTANTS_ANISO if n == 20 else W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 300 + n)
    rhs = np.random.default_rng(n + 7).standard_normal((3, P.ndof))
    r = torch.tensor(rhs, device="cuda", dtype=torch.float32)
    out = []
    try:
        for pz in (1, 0):
            rb.set_tuning(rb.TUNE_MG_PZ, pz)
            s = torch.empty_like(r)
            P.mg_apply(mu, r, s, precision=rb.FP32_IR)
            out.append(s.cpu().numpy())
    finally:
        rb.set_tuning(rb.TUNE_MG_PZ, 1)
    assert np.array_equal(out[0], out[1])
    assert np.all(np.isfinite(out[0])) and np.linalg.norm(out[0]) > 0


def test_refinement_fused_interpolation_same_bits(rb):
    """FP32 MGCG inside FP64 refinement on a batch of two grid sizes (40 and 72)
    gives the same iterations and solutions with and without the fused
    interpolation."""
    specs = [W.Problem(40, W.KIND_OCTANTS), W.Problem(72, W.KIND_OCTANTS)]
    probs = [rb.Problem(sp) for sp in specs]
    mus = [W.sample_mu(sp, 0.01, 100.0, 3, 400 + sp.n) for sp in specs]
    problem_of = np.array([0, 1, 1, 0, 1, 0], dtype=np.int32)
    cnt = [0, 0]
    mu = []
    for q in problem_of:
        mu.append(mus[q][cnt[q]])
        cnt[q] += 1
    mu = np.array(mu)
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=rb.PREC_MG, ir_mode=rb.IR_RELIABLE,
                           eta_inner=0.1, mg_omega=0.9)
    out = []
    try:
        for pz in (1, 0):
            rb.set_tuning(rb.TUNE_MG_PZ, pz)
            u = [torch.empty(probs[q].ndof, dtype=torch.float64, device="cuda") for q in problem_of]
            st = rb.solve(probs, mu, opts, problem_of=problem_of, u_out=u)
            out.append((st, [t.cpu().numpy() for t in u]))
    finally:
        rb.set_tuning(rb.TUNE_MG_PZ, 1)
    (s1, u1), (s0, u0) = out
    assert all(s["status"] == rb.SOLVE_CONVERGED for s in s1)
    assert [s["iters"] for s in s1] == [s["iters"] for s in s0]
    assert [s["outer_iters"] for s in s1] == [s["outer_iters"] for s in s0]
    assert all(np.array_equal(a, b) for a, b in zip(u1, u0))


def test_vcycle_operator_errors(rb):
    spec = W.Problem(8, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.1, 10.0, 1, 1)
    r = torch.zeros((1, P.ndof), dtype=torch.float64, device="cuda")
    for kw in ({"nu": 0}, {"nu": 9}, {"omega": 0.0}, {"omega": 1.5}):
        with pytest.raises(rb.RbwsError):
            P.mg_apply(mu, r, torch.empty_like(r), **kw)


def test_mgcg_forced_exact_dots_and_launches(rb):
    spec = W.Problem(15, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 8)
    x0, s0 = gpu_mgcg(rb, [P], mu, 1e-10)
    x1, s1 = gpu_mgcg(rb, [P], mu, 1e-10, flags=rb.FLAG_FORCE_EXACT_DOTS | rb.FLAG_NO_GRAPH)
    assert [s["iters"] for s in s0] == [s["iters"] for s in s1]
    for a, b in zip(x0, x1):
        assert np.array_equal(a, b)


def test_mgcg_rb_start_parity(rb):
    wl = W.blocks3_16()
    spec = wl.problem
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 64, W.SEED_TRAIN)
    gb = rb.Basis.build(P, mut, 10, wl.snap_tol, precond=rb.PREC_JACOBI)
    ob = oracle.greedy(O, mut, 10, wl.snap_tol, prec=oracle.PREC_JACOBI)
    mus = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 6, W.SEED_TEST)
    xg, sg = gpu_mgcg(rb, [P], mus, wl.tol, init=rb.INIT_RB, bases=[gb])
    for b in range(len(mus)):
        u0 = ob.lift(ob.coeffs(mus[b]))
        xo, so = O.mgcg(mus[b], u0=u0, tol=wl.tol)
        assert sg[b]["iters"] == so["iters"] and np.array_equal(xg[b], xo)


def test_mgcg_mixed_levels_batch(rb):
    """Grids with different numbers of levels in one launch (16: 3 levels, 20: 4, 9: 3)."""
    specs = [W.Problem(16, W.KIND_OCTANTS), W.Problem(20, W.KIND_OCTANTS), W.Problem(9, W.KIND_OCTANTS)]
    probs = [rb.Problem(s) for s in specs]
    assign = np.array([0, 1, 2, 1, 0, 2, 1], dtype=np.int32)
    mu = W.sample_mu(specs[0], 0.01, 100.0, len(assign), 77)
    xg, sg = gpu_mgcg(rb, probs, mu, 1e-10, problem_of=assign)
    for b, q in enumerate(assign):
        xo, so = oracle.Problem(specs[q]).mgcg(mu[b], tol=1e-10)
        assert sg[b]["iters"] == so["iters"] and np.array_equal(xg[b], xo)


def test_mgcg_64_sample(rb):
    spec = W.Problem(64, W.KIND_BLOCKS, W.BLOCKS4)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.1, 10.0, 8, W.SEED_TEST)
    xg, sg = gpu_mgcg(rb, [P], mu, 1e-10)
    O = oracle.Problem(spec)
    for b in (0, 5):
        xo, so = O.mgcg(mu[b], tol=1e-10)
        assert sg[b]["iters"] == so["iters"] and np.array_equal(xg[b], xo)


@pytest.mark.parametrize("n", [72, 70])
def test_mgcg_whole_row_tiles(rb, n):
    """Grids with 64 < n <= 128 run on 128 x 8 tiles that span the row (vector
    loads at n = 72, scalar row ends at n = 70; the coarse levels 35 and 34 on
    64 x 16 tiles): FP64 MGCG trajectories bitwise equal to the oracle's."""
    spec = W.Problem(n, W.KIND_OCTANTS)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 3, 70 + n)
    xg, sg = gpu_mgcg(rb, [P], mu, 1e-10)
    O = oracle.Problem(spec)
    xo, so = O.mgcg_batch(mu, tol=1e-10)
    for b in range(len(mu)):
        assert sg[b]["iters"] == so[b]["iters"] and sg[b]["final_rr"] == so[b]["final_rr"]
        assert np.array_equal(xg[b], xo[b])


def test_tile_depth_does_not_change_results(rb):
    """RBWS_TUNE_TZ fixes the tile depth; FP64 trajectories do not depend on it."""
    spec = W.Problem(40, W.KIND_BLOCKS, W.BLOCKS3)
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, 0.1, 10.0, 3, 5)
    out = []
    try:
        for tz in (4, 16, 64, 0):
            rb.set_tuning(rb.TUNE_TZ, tz)
            out.append(gpu_mgcg(rb, [P], mu, 1e-10))
    finally:
        rb.set_tuning(rb.TUNE_TZ, 0)
    x0, s0 = out[0]
    for x, st in out[1:]:
        assert [a["iters"] for a in st] == [a["iters"] for a in s0]
        assert all(np.array_equal(a, b) for a, b in zip(x, x0))
    with pytest.raises(rb.RbwsError):
        rb.set_tuning(rb.TUNE_TZ, 12)


@pytest.mark.parametrize("spec", [W.Problem(20, W.KIND_OCTANTS), W.Problem(33, W.KIND_BLOCKS, W.BLOCKS4)],
                         ids=["oct20", "blk33"])
@pytest.mark.parametrize("mode", [0, 1])
def test_refinement_with_multigrid(rb, spec, mode):
    """FP32 MGCG inside FP64 refinement: the solution matches the oracle's FP64
    reference to 1e-8, in about as many inner iterations as FP64 MGCG needs."""
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mu = W.sample_mu(spec, 0.01, 100.0, 6, 60 + spec.n)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mu))]
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=rb.PREC_MG, ir_mode=mode,
                           eta_inner=0.1 if mode == rb.IR_RELIABLE else 1e-4)
    st = rb.solve([P], mu, opts, u_out=u)
    torch.cuda.synchronize()
    ref, _ = O.cg_batch(mu, tol=1e-12, maxit=20000)
    _, so = O.mgcg_batch(mu, tol=1e-10)
    for b in range(len(mu)):
        assert st[b]["status"] == rb.SOLVE_CONVERGED
        assert st[b]["final_rr"] <= 1e-20 * st[b]["ff"]
        ub = u[b].cpu().numpy()
        assert np.linalg.norm(ub - ref[b]) <= 1e-8 * np.linalg.norm(ref[b])
        assert st[b]["iters"] <= 2 * so[b]["iters"] + 10, (st[b]["iters"], so[b]["iters"])


@pytest.mark.parametrize("eta,start", [(0.1, "zero"), (0.05, "rb")])
def test_refinement_with_multigrid_full_size_sample(rb, eta, start):
    """128^3, FP32 V-cycle CG inside FP64 refinement with reliable updates, on
    64 solves: the library default (inner tolerance 0.1, zero start) and the
    bench's launch configuration (tile depth 32, tolerance 0.05, RB start lifted
    on the matrix cores, from a small basis here); two sampled solutions against
    the oracle's FP64 MGCG solved to 1e-12."""
    wl = W.octants_128()
    spec = wl.problem
    P = rb.Problem(spec)
    mu = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 64, W.SEED_TEST)
    picks = (0, 37)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") if b in picks else None for b in range(len(mu))]
    kw, bases = {}, None
    if start == "rb":
        mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 64, W.SEED_TRAIN)
        bases = [rb.Basis.build(P, mut, 8, wl.snap_tol)]
        kw = dict(init=rb.INIT_RB, lift=rb.LIFT_MFMA)
    opts = rb.default_opts(tol=wl.tol, precision=rb.FP32_IR, precond=rb.PREC_MG, ir_mode=rb.IR_RELIABLE,
                           eta_inner=eta, mg_omega=0.9, **kw)
    try:
        if start == "rb":
            rb.set_tuning(rb.TUNE_TZ, 32)
        st = rb.solve([P], mu, opts, bases=bases, u_out=u)
        torch.cuda.synchronize()
    finally:
        rb.set_tuning(rb.TUNE_TZ, 0)
    assert all(s["status"] == rb.SOLVE_CONVERGED for s in st)
    assert all(s["final_rr"] <= wl.tol ** 2 * s["ff"] for s in st)
    if start == "rb":
        assert all(s["init_used"] == rb.INIT_RB for s in st)
    O = oracle.Problem(spec)
    for b in picks:
        ref, so = O.mgcg(mu[b], tol=1e-12)
        assert so["status"] == oracle.CONVERGED
        ub = u[b].cpu().numpy()
        assert np.linalg.norm(ub - ref) <= 1e-8 * np.linalg.norm(ref)
