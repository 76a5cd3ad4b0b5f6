"""The workloads at their full sizes, on the GPU, through the C ABI.

- blocks4-64 (64^3, four blocks, 512 training parameters, N = 30): the GPU
  greedy equals the oracle's, bit for bit, step by step (selected parameters,
  every indicator value, every basis vector, the reduced matrices).  The
  oracle's build takes about a quarter of an hour on eight cores, so its
  result is stored as digests in tests/golden/blocks4_64_greedy.json, written
  by tests/golden/make_blocks4_64_greedy.py, which calls only the oracle.
- octants8-128 (128^3, 1024 training parameters, N = 40, the benchmark's
  basis): the invariants the greedy and the Galerkin solve guarantee at any
  size (Alg. 4, Sec. 2.3), checked with the oracle's correctly rounded dots:
  an orthonormal V, each selected snapshot reproduced by its own reduced
  solve, Galerkin orthogonality of the reduced residual.
- the benchmark's launch configuration (1024 solves at 128^3 from the RB start,
  FP32 PCG with the V-cycle inside FP64 refinement, tile depth 32, inner
  tolerance 0.05, smoother weight 0.9, MFMA lift): every solve's true residual,
  recomputed from its returned solution, meets 1e-10, and sampled solutions
  match the oracle's FP64 MGCG to 1e-8.
"""
import concurrent.futures as cf
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2311_13862_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_64 = os.path.join(HERE, "golden", "blocks4_64_greedy.json")
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def rb():
    from paper_2311_13862_amd import rbws
    assert torch.cuda.is_available()
    return rbws


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def exact_dots_parallel(pairs, threads=16):
    """Correctly rounded dots (the oracle's) of many long vector pairs, in threads."""
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda xy: oracle.exact_dot(xy[0], xy[1]), pairs))


def test_greedy_blocks4_64_matches_stored_oracle(rb):
    with open(GOLDEN_64) as fh:
        g = json.load(fh)
    wl = W.blocks4_64()
    assert (g["n"], g["n_train"], g["N"], g["snap_tol"]) == (wl.problem.n, wl.n_train, wl.N, wl.snap_tol)
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    P = rb.Problem(wl.problem)
    gb = rb.Basis.build(P, mut, wl.N, wl.snap_tol, precond=rb.PREC_JACOBI)
    print("selected", list(gb.selected))
    assert gb.N == g["N_reached"]
    assert [int(s) for s in gb.selected] == g["selected"]
    V, A, f = gb.get()
    for k, st in enumerate(g["steps"]):
        assert float(gb.hist[k].max()).hex() == st["hist_max"], k
        assert sha(gb.hist[k]) == st["hist_sha256"], k
        assert [float(v).hex() for v in V[k][:4]] == st["v_head"], k
        assert sha(V[k]) == st["v_sha256"], k
    assert sha(A) == g["AqN_sha256"]
    assert sha(f) == g["fN_sha256"]


@pytest.fixture(scope="module")
def octants128(rb):
    wl = W.octants_128()
    spec = wl.problem
    mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    P = rb.Problem(spec)
    gb = rb.Basis.build(P, mut, wl.N, wl.snap_tol, precond=rb.PREC_JACOBI)
    return wl, spec, mut, P, gb


def test_octants128_basis_invariants(rb, octants128):
    wl, spec, mut, P, gb = octants128
    assert gb.N == wl.N
    V, A, fN = gb.get()
    N, nd = V.shape
    # orthonormality (CGS2), every entry of V^T V with correctly rounded dots
    pairs = [(V[i], V[j]) for i in range(N) for j in range(i, N)]
    G = exact_dots_parallel(pairs)
    k = 0
    worst = 0.0
    for i in range(N):
        for j in range(i, N):
            worst = max(worst, abs(G[k] - (1.0 if i == j else 0.0)))
            k += 1
    assert worst <= 1e-13, worst
    # the reduced matrices are symmetric
    for q in range(A.shape[0]):
        assert np.array_equal(A[q], A[q].T)
    # each selected snapshot is reproduced by its own reduced solve: u(mu_l) by the
    # greedy's own snapshot solver (Jacobi-PCG from zero to the snapshot tolerance)
    sel = np.asarray(gb.selected)
    mus = mut[sel]
    u = torch.empty((len(sel), nd), dtype=torch.float64, device="cuda")
    st = rb.solve([P], mus, rb.default_opts(tol=wl.snap_tol, precond=rb.PREC_JACOBI),
                  u_out=[u[b] for b in range(len(sel))])
    assert np.all(st["status"] == rb.SOLVE_CONVERGED)
    c = gb.coeffs(mus)
    cd = torch.from_numpy(c).cuda()
    ul = torch.empty_like(u)
    gb.lift(cd, ul, mode=rb.LIFT_EXACT)
    torch.cuda.synchronize()
    rel = (torch.linalg.vector_norm(ul - u, dim=1) / torch.linalg.vector_norm(u, dim=1)).cpu().numpy()
    print(f"snapshots reproduced to {rel.max():.2e}")
    assert rel.max() <= 1e-10, rel.max()
    # the greedy's indicator at a selected parameter, ||f - A V c|| / ||f||, is at most the
    # snapshot's own relative residual (<= the snapshot tolerance) plus ||A (V c - u)|| / ||f||:
    # at this contrast (1e4) and size a reproduction error of 1e-13 moves the residual by
    # up to cond(A) times as much, so the bound is computed, not fixed
    h2 = 1.0 / (spec.n + 1) ** 2
    fnorm = h2 * np.sqrt(nd)
    adiff = torch.empty_like(u)
    P.spmv(mus, ul - u, adiff)
    torch.cuda.synchronize()
    rdiff = (torch.linalg.vector_norm(adiff, dim=1) / fnorm).cpu().numpy()
    # each residual evaluation r = f - A x rounds by at most 8 eps (|f| + |A| |x|) per
    # entry, and || |A| x || <= 2 max_P d_P ||x|| with d_P <= 6 max(mu)
    unorm = torch.linalg.vector_norm(u, dim=1).cpu().numpy()
    rnd = 3 * 8 * EPS * (1.0 + 12.0 * mus.max(axis=1) * unorm / fnorm)
    last = gb.hist[-1]
    print(f"indicator at the selected parameters: max {last[sel].max():.2e}; "
          f"||A (V c - u)|| / ||f||: max {rdiff.max():.2e}; rounding bound: max {rnd.max():.2e}")
    assert np.all(last[sel] <= wl.snap_tol + rdiff + rnd), (last[sel], rdiff, rnd)
    assert np.all(last[sel] <= 1e-6 * last.max())
    del u, ul, adiff
    # Galerkin orthogonality: V^T (f - A(mu) V c(mu)) = f_N - A_N(mu) c(mu), zero up to
    # the rounding of the reduced solve, the lift and the residual
    mut8 = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 8, W.SEED_TEST)
    c8 = gb.coeffs(mut8)
    u0 = torch.empty((8, nd), dtype=torch.float64, device="cuda")
    gb.lift(torch.from_numpy(c8).cuda(), u0, mode=rb.LIFT_EXACT)
    au = torch.empty_like(u0)
    P.spmv(mut8, u0, au)
    torch.cuda.synchronize()
    r0 = (h2 - au).cpu().numpy()
    th = P.theta(mut8)
    for b in range(8):
        vr = np.array(exact_dots_parallel([(V[i], r0[b]) for i in range(N)]))
        AN = np.einsum("q,qij->ij", th[b], A)
        bound = 1e-12 * fnorm + 64 * EPS * np.linalg.norm(AN, 2) * np.linalg.norm(c8[b])
        print(f"mu {b}: ||V^T r0|| / ||f|| = {np.linalg.norm(vr) / fnorm:.3e}")
        assert np.linalg.norm(vr) <= bound, (b, np.linalg.norm(vr) / fnorm)


def test_bench_configuration_parity(rb, octants128):
    """The benchmark's timed step, at its size and in its launch configuration."""
    wl, spec, mut, P, gb = octants128
    mu = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    nd = P.ndof
    rb.set_tuning(rb.TUNE_TZ, 32)
    try:
        u = torch.empty((len(mu), nd), dtype=torch.float64, device="cuda")
        opts = rb.default_opts(precision=rb.FP32_IR, tol=wl.tol, precond=rb.PREC_MG, eta_inner=0.05,
                               init=rb.INIT_RB, lift=rb.LIFT_MFMA, ir_mode=rb.IR_RELIABLE, mg_omega=0.9)
        st = rb.solve([P], mu, opts, bases=[gb], u_out=[u[b] for b in range(len(mu))])
        torch.cuda.synchronize()
    finally:
        rb.set_tuning(rb.TUNE_TZ, 0)
    assert np.all(st["status"] == rb.SOLVE_CONVERGED)
    assert np.all(st["final_rr"] <= wl.tol ** 2 * st["ff"])
    # the true residual of every returned solution, recomputed in FP64 (chunks of 128 solves)
    h2 = 1.0 / (spec.n + 1) ** 2
    fnorm = h2 * np.sqrt(nd)
    worst = 0.0
    for b0 in range(0, len(mu), 128):
        au = torch.empty((128, nd), dtype=torch.float64, device="cuda")
        P.spmv(mu[b0:b0 + 128], u[b0:b0 + 128], au)
        rel = (torch.linalg.vector_norm(h2 - au, dim=1) / fnorm).cpu().numpy()
        worst = max(worst, float(rel.max()))
        del au
    assert worst <= 1.0000001e-10, worst
    # sampled solutions against the oracle's FP64 MGCG (same V-cycle, omega 0.9) to 1e-12
    pick = [0, 333, 777, 1023]
    O = oracle.Problem(spec)
    ref, so = O.mgcg_batch(mu[pick], tol=1e-12, omega=0.9, nthreads=4)
    for k, b in enumerate(pick):
        assert so[k]["status"] == 0
        ub = u[b].cpu().numpy()
        err = np.linalg.norm(ub - ref[k]) / np.linalg.norm(ref[k])
        print(f"solve {b}: relative error vs the oracle {err:.2e}")
        assert err <= 1e-8, (b, err)
