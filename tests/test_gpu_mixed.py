"""The anisotropic workload with the parameter-dependent Gaussian source, and
uneven batches that mix grid sizes in one launch, against the CPU oracle.

Both sides evaluate the source's exponential rounded to nearest (the GPU in
double-double arithmetic, the oracle through binary128), so f_h is the same
on both and FP64 CG from zero matches bit for bit.  The reduced right-hand
side V^T f(mu) is an FP64 matrix-core contraction on the GPU (with the device
library's exp) and a correctly rounded projection in the oracle, so the
greedy, the RB coefficients and RB-started solves are compared to tolerances
(iteration counts within a few, solutions to 1e-9 in FP64, 1e-8 after
refinement)."""
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


def gauss_spec(n):
    return W.Problem(n, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02)


@pytest.fixture(scope="module")
def mixed(rb):
    """Per-size greedy bases (N = 8 from 40 training parameters) on 12^3, 16^3, 21^3."""
    out = []
    for n in (12, 16, 21):
        spec = gauss_spec(n)
        mut = W.sample_mu(spec, 0.1, 10.0, 40, W.SEED_TRAIN + 10 * n)
        P = rb.Problem(spec)
        gb = rb.Basis.build(P, mut, 8, 1e-12)
        O = oracle.Problem(spec)
        ob = oracle.greedy(O, mut, 8, 1e-12, prec=oracle.PREC_JACOBI)
        out.append((spec, mut, P, gb, O, ob))
    return out


def test_gauss_greedy_matches_oracle(rb, mixed):
    for spec, mut, P, gb, O, ob in mixed:
        assert gb.N == ob.N == 8
        # the indicator at each step must not be a near-tie for the selection to be comparable
        for k in range(gb.N - 1):
            row = np.sort(ob.hist[k])[::-1]
            assert row[0] > row[1] * (1 + 1e-6), (spec.n, k)
        assert list(gb.selected) == list(ob.selected)
        # entries at selected parameters sit at the snapshot tolerance (~1e-12): absolute there
        np.testing.assert_allclose(gb.hist, ob.hist, rtol=1e-7, atol=1e-10)
        V, A, _ = gb.get()
        assert np.abs(V - ob.V).max() <= 1e-9
        np.testing.assert_allclose(A, ob.AqN[:, :8, :8], rtol=1e-9, atol=1e-12 * np.abs(ob.AqN).max())


@pytest.mark.parametrize("prec", [0, 1])
def test_gauss_fp64_cg_bitwise(rb, prec):
    """FP64 PCG from zero (P = I and Jacobi) on the Gaussian-source problem at
    21^3: iteration counts, residuals and solutions equal to the oracle's."""
    spec = gauss_spec(21)
    P = rb.Problem(spec)
    O = oracle.Problem(spec)
    mus = W.sample_mu(spec, 0.1, 10.0, 6, 77)
    u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
    st = rb.solve([P], mus, rb.default_opts(tol=1e-10, precond=prec), u_out=u)
    torch.cuda.synchronize()
    for b, m in enumerate(mus):
        xo, so = O.cg(m, prec=prec, tol=1e-10)
        assert st[b]["ff"] == so["ff"] and st[b]["init_rr"] == so["init_rr"], b
        assert st[b]["iters"] == so["iters"] and st[b]["final_rr"] == so["final_rr"], b
        assert np.array_equal(u[b].cpu().numpy(), xo), b


def test_gauss_online_coeffs(rb, mixed):
    for spec, mut, P, gb, O, ob in mixed:
        mus = W.sample_mu(spec, 0.1, 10.0, 10, W.SEED_TEST + spec.n)
        c = gb.coeffs(mus)
        for b in range(len(mus)):
            co = ob.coeffs(mus[b])
            assert np.linalg.norm(c[b] - co) <= 1e-9 * np.linalg.norm(co)


@pytest.mark.parametrize("precision", ["fp64", "fp32ir"])
def test_mixed_batch(rb, mixed, precision):
    probs = [m[2] for m in mixed]
    bases = [m[3] for m in mixed]
    nsol = 12
    assign = np.arange(nsol, dtype=np.int32) % 3
    mus = np.concatenate([W.sample_mu(mixed[q][0], 0.1, 10.0, 1, 100 + i) for i, q in enumerate(assign)])
    u = [torch.empty(probs[q].ndof, dtype=torch.float64, device="cuda") for q in assign]
    prec = rb.FP64 if precision == "fp64" else rb.FP32_IR
    tol = 1e-10
    for init in (rb.INIT_ZERO, rb.INIT_RB):
        st = rb.solve(probs, mus, rb.default_opts(tol=tol, precision=prec, init=init), problem_of=assign,
                      bases=bases, u_out=u)
        torch.cuda.synchronize()
        lat = [s["t_done_ms"] for s in st]
        assert all(s["status"] == rb.SOLVE_CONVERGED for s in st)
        assert all(t > 0 for t in lat)
        for b, q in enumerate(assign):
            O = mixed[q][4]
            if init == rb.INIT_ZERO:
                xo, so = O.cg(mus[b], tol=tol)
            else:
                xo, so, _ = oracle.rbi_cg(mixed[q][5], mus[b], tol=tol)
            ub = u[b].cpu().numpy()
            if precision == "fp64" and init == rb.INIT_ZERO:
                # the same f_h, the same algorithm from zero: bit for bit
                assert st[b]["iters"] == so["iters"], (b, st[b]["iters"], so["iters"])
                assert st[b]["final_rr"] == so["final_rr"]
                assert np.array_equal(ub, xo), b
            elif precision == "fp64":
                # from the RB start: the starts differ in the projection's last bits
                assert abs(st[b]["iters"] - so["iters"]) <= 2, (b, st[b]["iters"], so["iters"])
                rel = np.linalg.norm(ub - xo) / np.linalg.norm(xo)
                assert rel <= 1e-9, rel
            else:
                ref, _ = O.cg(mus[b], tol=1e-13)
                rel = np.linalg.norm(ub - ref) / np.linalg.norm(ref)
                assert rel <= 1e-8, rel
            assert st[b]["final_rr"] <= tol * tol * st[b]["ff"]


def test_aniso_mixed_full_sizes(rb):
    """The anisotropic workload's uneven batch at its real grid sizes: 24 solves,
    solve i on 64^3, 96^3 or 128^3 (i mod 3), in one launch, FP32 PCG with the
    V-cycle inside FP64 refinement from per-size RB starts (small bases: N = 8
    from 32 training parameters).  One solve per size against the oracle's FP64
    MGCG to 1e-8; every solve's recursive and device-clock statistics valid."""
    sizes = (64, 96, 128)
    probs, bases, specs = [], [], []
    for q, n in enumerate(sizes):
        spec = gauss_spec(n)
        mut = W.sample_mu(spec, 0.1, 10.0, 32, W.SEED_TRAIN + 10 * q)
        P = rb.Problem(spec)
        probs.append(P)
        bases.append(rb.Basis.build(P, mut, 8, 1e-12))
        specs.append(spec)
    nsol = 24
    assign = (np.arange(nsol) % 3).astype(np.int32)
    mus = np.empty((nsol, specs[0].p))
    for q in range(3):
        mus[assign == q] = W.sample_mu(specs[q], 0.1, 10.0, int(np.sum(assign == q)), W.SEED_TEST + 10 * q)
    u = [torch.empty(probs[q].ndof, dtype=torch.float64, device="cuda") for q in assign]
    opts = rb.default_opts(tol=1e-10, precision=rb.FP32_IR, precond=rb.PREC_MG, init=rb.INIT_RB,
                           lift=rb.LIFT_MFMA, eta_inner=0.05, mg_omega=0.9, ir_mode=rb.IR_RELIABLE)
    st = rb.solve(probs, mus, opts, problem_of=assign, bases=bases, u_out=u)
    torch.cuda.synchronize()
    assert np.all(st["status"] == rb.SOLVE_CONVERGED)
    assert np.all(st["final_rr"] <= 1e-20 * st["ff"])
    assert np.all(st["t_done_ms"] > 0)
    # one solve per size (the first of each) against the oracle's FP64 MGCG
    import concurrent.futures as cf

    def ref(q):
        b = int(np.flatnonzero(assign == q)[0])
        O = oracle.Problem(specs[q])
        x, s = O.mgcg(mus[b], tol=1e-12, omega=0.9)
        return b, x, s

    with cf.ThreadPoolExecutor(3) as ex:
        for b, x, s in ex.map(ref, range(3)):
            assert s["status"] == 0
            ub = u[b].cpu().numpy()
            err = np.linalg.norm(ub - x) / np.linalg.norm(x)
            print(f"solve {b} at {specs[assign[b]].n}^3: error vs the oracle {err:.2e}, "
                  f"{st[b]['iters']} inner / {st[b]['outer_iters']} outer iterations")
            assert err <= 1e-8, (b, err)
