"""GPU parity of the reduced basis (Alg. 4 skeleton, Eq. "RB system",
Alg. 5) against the CPU oracle, through the C ABI.

The greedy build, the online Galerkin solve and the exact lift use correctly
rounded inner products on both sides, so the GPU selects the same training
parameters and produces the same basis, reduced matrices, indicators, RB
coefficients, warm starts, iteration counts and solutions, bit for bit.
"""
import os

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


@pytest.fixture(scope="module")
def c1(rb):
    wl = W.blocks3_16()
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    O = oracle.Problem(wl.problem)
    ob = oracle.greedy(O, mut, wl.N, wl.snap_tol, prec=oracle.PREC_JACOBI)
    P = rb.Problem(wl.problem)
    gb = rb.Basis.build(P, mut, wl.N, wl.snap_tol, precond=rb.PREC_JACOBI)
    return wl, mut, O, ob, P, gb


def test_greedy_parity(c1):
    wl, mut, O, ob, P, gb = c1
    assert gb.N == ob.N == wl.N
    assert list(gb.selected) == list(ob.selected)
    assert np.array_equal(gb.hist, ob.hist)
    V, A, f = gb.get()
    assert np.array_equal(V, ob.V)
    assert np.array_equal(A, ob.AqN[:, :gb.N, :gb.N])
    assert np.array_equal(f, ob.fN[:gb.N])
    assert gb.final_max == ob.hist[-1].max()


def test_online_coeffs_and_lift(rb, c1):
    wl, mut, O, ob, P, gb = c1
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    c = gb.coeffs(mus)
    for b in range(len(mus)):
        assert np.array_equal(c[b], ob.coeffs(mus[b]))
    cd = torch.from_numpy(c).cuda()
    u = torch.empty((len(mus), P.ndof), dtype=torch.float64, device="cuda")
    gb.lift(cd, u, mode=rb.LIFT_EXACT)
    um = torch.empty_like(u)
    gb.lift(cd, um, mode=rb.LIFT_MFMA)
    torch.cuda.synchronize()
    u, um = u.cpu().numpy(), um.cpu().numpy()
    for b in range(len(mus)):
        ue = ob.lift(c[b])
        assert np.array_equal(u[b], ue)
        assert np.abs(um[b] - ue).max() <= 1e-14 * np.abs(ue).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_warm_start_parity(rb, c1, prec):
    wl, mut, O, ob, P, gb = c1
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
    opts = rb.default_opts(tol=wl.tol, precond=prec, init=rb.INIT_RB, lift=rb.LIFT_EXACT)
    sg = rb.solve([P], mus, opts, bases=[gb], u_out=u)
    zg = rb.solve([P], mus, rb.default_opts(tol=wl.tol, precond=prec))
    torch.cuda.synchronize()
    for b, m in enumerate(mus):
        xo, so, _ = oracle.rbi_cg(ob, m, prec=prec, tol=wl.tol)
        assert sg[b]["iters"] == so["iters"] and sg[b]["extra_spmv"] == so["extra_spmv"]
        assert sg[b]["init_rr"] == so["init_rr"] and sg[b]["final_rr"] == so["final_rr"]
        assert np.array_equal(u[b].cpu().numpy(), xo)
        assert sg[b]["iters"] <= zg[b]["iters"]          # warm <= zero (paper, Sec. 4)


def test_basis_save_load(rb, c1, tmp_path):
    wl, mut, O, ob, P, gb = c1
    path = str(tmp_path / "basis.bin")
    gb.save(path)
    lb = rb.Basis.load(P, path)
    assert lb.N == gb.N and lb.final_max == gb.final_max
    for a, b in zip(lb.get(), gb.get()):
        assert np.array_equal(a, b)
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 4, W.SEED_TEST)
    assert np.array_equal(lb.coeffs(mus), gb.coeffs(mus))
    other = rb.Problem(W.Problem(16, W.KIND_OCTANTS))
    with pytest.raises(rb.RbwsError):
        rb.Basis.load(other, path)


def test_greedy_parity_ragged_40(rb):
    # 40^3 grid (ragged tiles), four blocks, small training set
    spec = W.Problem(40, W.KIND_BLOCKS, W.BLOCKS4)
    mut = W.sample_mu(spec, 0.1, 10.0, 24, W.SEED_TRAIN)
    O = oracle.Problem(spec)
    ob = oracle.greedy(O, mut, 5, 1e-12, prec=oracle.PREC_JACOBI)
    P = rb.Problem(spec)
    gb = rb.Basis.build(P, mut, 5, 1e-12, precond=rb.PREC_JACOBI)
    assert list(gb.selected) == list(ob.selected)
    assert np.array_equal(gb.hist, ob.hist)
    V, A, f = gb.get()
    assert np.array_equal(V, ob.V) and np.array_equal(A, ob.AqN)
    mus = W.sample_mu(spec, 0.1, 10.0, 3, W.SEED_TEST)
    opts = rb.default_opts(tol=1e-10, precond=1, init=rb.INIT_RB)
    sg = rb.solve([P], mus, opts, bases=[gb])
    for b, m in enumerate(mus):
        _, so, _ = oracle.rbi_cg(ob, m, prec=1, tol=1e-10)
        assert sg[b]["iters"] == so["iters"] and sg[b]["final_rr"] == so["final_rr"]


def test_rb_errors(rb, c1):
    wl, mut, O, ob, P, gb = c1
    with pytest.raises(rb.RbwsError) as e:
        rb.solve([P], mut[:2], rb.default_opts(init=rb.INIT_RB))
    assert e.value.code == rb.ESTATE
    with pytest.raises(rb.RbwsError) as e:
        rb.Basis.build(P, mut[:3], 5, 1e-12)
    assert e.value.code == rb.EINVAL
    with pytest.raises(rb.RbwsError) as e:
        gb.coeffs(-np.ones((1, 3)))                    # indefinite reduced matrix
    assert e.value.code == rb.ENUMERIC
