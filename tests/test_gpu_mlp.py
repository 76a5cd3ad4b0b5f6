"""GPU parity of the learned start (a BF16-MFMA perceptron mu -> c(mu), an
addition to the paper's Alg. 5 initial value) against the FP64 oracle
(oracle/mlp.py), through the C ABI.

Weights are drawn here from a seeded generator and handed to both sides.
The GPU rounds weights and activations to bfloat16 (8 significant bits) and
accumulates in FP32, so outputs and gradients are compared per tensor by
relative error (<= 2e-2) and cosine (>= 0.999).  Adam is compared on the
GPU's own gradient (FP32 arithmetic on both sides of the same input)."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2311_13862_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, COS = 2e-2, 0.999


@pytest.fixture(scope="module")
def rb():
    from paper_2311_13862_amd import rbws
    assert torch.cuda.is_available()
    return rbws


def init_params(rng, p, nout, hidden, depth):
    layers = []
    for l in range(depth + 1):
        i = p if l == 0 else hidden
        o = nout if l == depth else hidden
        W_ = rng.uniform(-1.0, 1.0, (o, i)) / math.sqrt(i)
        b_ = 0.1 * rng.standard_normal(o)
        layers.append((W_.astype(np.float32).astype(np.float64), b_.astype(np.float32).astype(np.float64)))
    return layers


def close(a, b, rel=REL, cos=COS):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    err = np.linalg.norm(a - b) / nb
    c = float(a @ b / (np.linalg.norm(a) * nb))
    return err <= rel and c >= cos, (err, c)


def octant_case(rb, nrows, seed=11, hidden=256, depth=3, nout=40):
    spec = W.Problem(16, W.KIND_OCTANTS)
    mu = W.sample_mu(spec, 0.01, 100.0, nrows, seed)
    rng = np.random.default_rng(W.SEED_MLP_INIT)
    layers = init_params(rng, 8, nout, hidden, depth)
    net = rb.Mlp.create(8, nout, hidden=hidden, depth=depth, log_cols=8, in_m=0.0, in_s=2.0,
                        params=rb.pack_params(layers))
    x = omlp.scale_inputs(mu, 8, m=0.0, s=2.0)
    return mu, layers, net, x


@pytest.mark.parametrize("nrows", [64, 37, 1])
def test_forward_parity(rb, nrows):
    mu, layers, net, x = octant_case(rb, nrows)
    y = net.forward(mu)
    yo, _ = omlp.forward(layers, x)
    ok, info = close(y, yo)
    assert ok, info
    # params round-trip exactly (FP32 masters)
    assert np.array_equal(net.get_params(), rb.pack_params(layers).astype(np.float32))


def test_gradient_parity(rb):
    mu, layers, net, x = octant_case(rb, 200, seed=12)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((200, 40))
    loss, g = net.grad(mu, c)
    lo, grads, _ = omlp.loss_and_grads(layers, x, c)
    assert abs(loss - lo) <= 2e-2 * lo, (loss, lo)
    gl = rb.unpack_params(g, 8, 40, 256, 3)
    for l, ((dW, db), (oW, ob)) in enumerate(zip(gl, grads)):
        ok, info = close(dW, oW)
        assert ok, ("dW", l, info)
        ok, info = close(db, ob)
        assert ok, ("db", l, info)
    # the gradient call does not change the parameters
    assert np.array_equal(net.get_params(), rb.pack_params(layers).astype(np.float32))


def test_adam_step(rb):
    mu, layers, net, x = octant_case(rb, 96, seed=13, hidden=64, depth=2, nout=12)
    c = np.random.default_rng(6).standard_normal((96, 12))
    p0 = net.get_params().astype(np.float64)
    _, g = net.grad(mu, c)
    lr = 1e-3
    net.adam_step(mu, c, lr)
    p1 = net.get_params().astype(np.float64)
    # the oracle's Adam on the same gradient (first step, bias-corrected)
    P = [p0.copy()]
    G = [g.astype(np.float64)]
    m = [np.zeros_like(p0)]
    v = [np.zeros_like(p0)]
    omlp.adam_step([(P[0], np.zeros(0))], [(G[0], np.zeros(0))], [(m[0], np.zeros(0))],
                   [(v[0], np.zeros(0))], 1, lr)
    # FP32 Adam: beta2 = 0.999 rounds to float (relative 1.3e-8), so 1 - beta2 is
    # off by 1.3e-5 relative and every update by about 6e-6 lr
    np.testing.assert_allclose(p1, P[0], rtol=2.0 ** -22, atol=2e-5 * lr)
    # a second step continues the moments (t = 2)
    _, g2 = net.grad(mu, c)
    net.adam_step(mu, c, lr)
    omlp.adam_step([(P[0], np.zeros(0))], [(g2.astype(np.float64), np.zeros(0))], [(m[0], np.zeros(0))],
                   [(v[0], np.zeros(0))], 2, lr)
    np.testing.assert_allclose(net.get_params(), P[0], rtol=2.0 ** -21, atol=4e-5 * lr)


def test_train_graph_equals_launches_and_learns(rb):
    spec = W.Problem(16, W.KIND_OCTANTS)
    mu = W.sample_mu(spec, 0.01, 100.0, 512, 21)
    # a smooth target of the scaled inputs
    x = omlp.scale_inputs(mu, 8, m=0.0, s=2.0)
    c = np.stack([np.sin(x @ np.linspace(0.1, 0.8, 8) * (j + 1) / 4) for j in range(8)], axis=1)
    nets = []
    hists = []
    for g in (False, True):
        net = rb.Mlp.create(8, 8, hidden=64, depth=2, log_cols=8, in_m=0.0, in_s=2.0, seed=7)
        h = net.train(mu, c, epochs=3, batch=64, lr=3e-3, seed=9, use_graph=g)
        h2 = net.train(mu, c, epochs=2, batch=64, lr=3e-3, seed=10, use_graph=g)
        nets.append(net)
        hists.append(np.concatenate([h, h2]))
    assert np.array_equal(nets[0].get_params(), nets[1].get_params())
    assert np.array_equal(hists[0], hists[1])  # every replayed step's loss
    assert len(hists[0]) == 5 * 8
    assert hists[0][-8:].mean() < 0.5 * hists[0][:8].mean()


def test_output_scaling_and_predict(rb):
    spec = W.Problem(16, W.KIND_OCTANTS)
    mu = W.sample_mu(spec, 0.01, 100.0, 300, 22)
    rng = np.random.default_rng(8)
    c = rng.standard_normal((300, 6)) * 5 + 2
    net = rb.Mlp.create(8, 6, hidden=32, depth=1, log_cols=8, in_m=0.0, in_s=2.0, out_pow=1.0, seed=3)
    net.fit_output_scaling(mu, c)
    mean, sd = net.output_scaling()
    t = c * 10.0 ** np.log10(mu).mean(axis=1, keepdims=True)
    np.testing.assert_allclose(mean, t.mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sd, t.std(axis=0), rtol=1e-12)
    y = net.forward(mu[:20]).astype(np.float64)
    pred = net.predict(mu[:20])
    ref = (mean + sd * y) * 10.0 ** (-np.log10(mu[:20]).mean(axis=1, keepdims=True))
    np.testing.assert_allclose(pred, ref, rtol=1e-6)


def test_save_load(rb, tmp_path):
    net = rb.Mlp.create(3, 5, hidden=32, depth=2, log_cols=3, seed=4)
    net.set_output_scaling([1, 2, 3, 4, 5], [1, 1, 2, 2, 3])
    path = str(tmp_path / "net.bin")
    net.save(path)
    n2 = rb.Mlp.load(path)
    assert np.array_equal(n2.get_params(), net.get_params())
    mu = np.exp(np.random.default_rng(0).uniform(-1, 1, (9, 3)))
    assert np.array_equal(n2.predict(mu), net.predict(mu))


def test_mlp_errors(rb):
    with pytest.raises(rb.RbwsError):
        rb.Mlp.create(3, 5, hidden=30)          # not a multiple of 32
    with pytest.raises(rb.RbwsError):
        rb.Mlp.create(3, 65)                    # too many outputs
    net = rb.Mlp.create(3, 5, hidden=32, depth=1, log_cols=3)
    with pytest.raises(rb.RbwsError):
        net.predict(np.array([[1.0, -1.0, 1.0]]))  # log of a negative parameter
    with pytest.raises(rb.RbwsError):
        net.train(np.ones((4, 3)), np.zeros((4, 5)), epochs=1, batch=8)


@pytest.fixture(scope="module")
def learned16(rb):
    """blocks3-16: greedy basis (N = 20), MLP trained on 2048 RB pairs."""
    wl = W.blocks3_16()
    spec = wl.problem
    P = rb.Problem(spec)
    mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    basis = rb.Basis.build(P, mut, wl.N, wl.snap_tol)
    mup = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 2048, W.SEED_MLP_PAIRS)
    c = basis.coeffs(mup)
    net = rb.Mlp.create(3, basis.N, hidden=128, depth=3, log_cols=3, in_m=0.0, in_s=1.0, seed=W.SEED_MLP_INIT)
    net.fit_output_scaling(mup, c)
    hist = net.train(mup, c, epochs=150, batch=128, lr=2e-3, lr_min=1e-5, seed=1)
    return wl, P, basis, net, hist


def test_learned_start_gain(rb, learned16):
    wl, P, basis, net, hist = learned16
    assert hist[-16:].mean() < 0.05 * hist[:16].mean()
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    # the network's coefficients against the reduced solve's
    c_rb = basis.coeffs(mus)
    c_nn = net.predict(mus)
    err = np.linalg.norm(c_nn - c_rb, axis=1) / np.linalg.norm(c_rb, axis=1)
    assert np.median(err) < 0.05, err
    runs = {}
    for name, init, fb in (("zero", rb.INIT_ZERO, 0), ("rb", rb.INIT_RB, 0),
                           ("learned", rb.INIT_LEARNED, 1), ("strict", rb.INIT_LEARNED, 0)):
        u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
        st = rb.solve([P], mus, rb.default_opts(tol=wl.tol, init=init, fallback=fb), bases=[basis],
                      mlps=[net], u_out=u)
        assert all(s["status"] == rb.SOLVE_CONVERGED for s in st)
        runs[name] = (st, u)
    it = {k: np.mean([s["iters"] for s in v[0]]) for k, v in runs.items()}
    # what the network gains over the zero start, at the same tolerance
    assert it["learned"] < it["zero"], it
    # and over the method without it (the RB start): iterations, the start stage's
    # time per batch (reduced solves against network inference), and throughput of
    # the whole solve, timed in interleaved rounds
    import time
    t_stage = {}
    for name, fn in (("rb_coeffs", lambda: basis.coeffs(mus)), ("mlp_predict", lambda: net.predict(mus))):
        fn()
        t = time.perf_counter()
        for _ in range(5):
            fn()
        t_stage[name] = (time.perf_counter() - t) / 5 * 1e3
    secs = {k: [] for k in ("rb", "strict", "zero")}
    opt = {"rb": rb.default_opts(tol=wl.tol, init=rb.INIT_RB),
           "strict": rb.default_opts(tol=wl.tol, init=rb.INIT_LEARNED, fallback=0),
           "zero": rb.default_opts(tol=wl.tol)}
    for _ in range(3):
        for k in secs:
            torch.cuda.synchronize()
            t = time.perf_counter()
            rb.solve([P], mus, opt[k], bases=[basis], mlps=[net])
            torch.cuda.synchronize()
            secs[k].append(time.perf_counter() - t)
    thr = {k: len(mus) / float(np.median(v)) for k, v in secs.items()}
    print("learned start vs RB start at blocks3-16:",
          {"inner_iters_mean": {k: float(v) for k, v in it.items()},
           "iters_gain_over_rb": {"cheap": float(it["rb"] - it["learned"]), "strict": float(it["rb"] - it["strict"])},
           "start_stage_ms_per_batch": t_stage,
           "mu_solves_per_s": thr, "strict_over_rb": thr["strict"] / thr["rb"],
           "started_from_mlp_strict": int(sum(s["init_used"] == rb.INIT_LEARNED for s in runs["strict"][0]))})
    # strict fallback: each solve starts from the smaller of the two true residuals
    for s_strict, s_l, s_r in zip(runs["strict"][0], runs["learned"][0], runs["rb"][0]):
        if s_l["init_used"] == rb.INIT_LEARNED:
            cand = s_l["init_rr"]
        else:
            cand = None
        # (the rule compares residual norms from the basis's decomposition: equal to the
        # true ones up to rounding, so a near-tie may go either way)
        assert s_strict["init_rr"] <= s_r["init_rr"] * (1 + 1e-9)
        if cand is not None:
            assert s_strict["init_rr"] <= cand * (1 + 1e-9)
    # solutions agree with the oracle's FP64 reference
    O = oracle.Problem(wl.problem)
    ref, _ = O.cg_batch(mus[:4], tol=1e-13)
    for name in runs:
        for b in range(4):
            ub = runs[name][1][b].cpu().numpy()
            assert np.linalg.norm(ub - ref[b]) <= 1e-9 * np.linalg.norm(ref[b]), name


def test_residual_estimate_matches_oracle(rb, learned16):
    """The basis's residual decomposition against the oracle's f - A(mu) V c,
    formed explicitly on the oracle's own greedy basis (the same selection),
    for the reduced solution, a perturbed one (the size of a network's error)
    and random coefficients."""
    wl, P, basis, net, hist = learned16
    spec = wl.problem
    O = oracle.Problem(spec)
    mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    ob = oracle.greedy(O, mut, wl.N, wl.snap_tol)
    assert list(basis.selected) == list(ob.selected)
    mus = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, 12, W.SEED_TEST + 3)
    rng = np.random.default_rng(3)
    c_rb = np.stack([ob.coeffs(m) for m in mus])
    for c in (c_rb, c_rb * (1.0 + 0.05 * rng.standard_normal(c_rb.shape)), rng.standard_normal(c_rb.shape)):
        est = basis.residual_estimate(mus, c)
        ref = []
        for m, cm in zip(mus, c):
            f = O.rhs(m)
            ref.append(np.linalg.norm(f - O.apply(m, ob.lift(cm))) / np.linalg.norm(f))
        np.testing.assert_allclose(est, ref, rtol=1e-8)


def test_strict_rule_decomposition_equals_explicit(rb, learned16):
    """The strict learned-start rule gives the same starts, trajectories and
    solutions whether the two residual norms come from the decomposition or
    from explicit FP64 residuals."""
    wl, P, basis, net, hist = learned16
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 24, W.SEED_TEST + 5)
    out = []
    for flags in (0, rb.FLAG_EXPLICIT_FALLBACK):
        u = [torch.empty(P.ndof, dtype=torch.float64, device="cuda") for _ in range(len(mus))]
        st = rb.solve([P], mus, rb.default_opts(tol=wl.tol, init=rb.INIT_LEARNED, fallback=0, flags=flags),
                      bases=[basis], mlps=[net], u_out=u)
        out.append((st, [t.cpu().numpy() for t in u]))
    (s0, u0), (s1, u1) = out
    assert [s["init_used"] for s in s0] == [s["init_used"] for s in s1]
    assert [s["iters"] for s in s0] == [s["iters"] for s in s1]
    assert all(np.array_equal(a, b) for a, b in zip(u0, u1))


def test_residual_estimate_needs_decomposition(rb):
    spec = W.Problem(8, W.KIND_OCTANTS_ANISO, (), W.F_GAUSS, 0.02)
    P = rb.Problem(spec)
    mut = W.sample_mu(spec, 0.1, 10.0, 8, 1)
    basis = rb.Basis.build(P, mut, 3, 1e-12)
    with pytest.raises(rb.RbwsError) as e:
        basis.residual_estimate(mut[:2], np.zeros((2, basis.N)))
    assert e.value.code == rb.ESTATE


def test_learned_start_needs_network(rb, learned16):
    wl, P, basis, net, hist = learned16
    mus = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, 2, W.SEED_TEST)
    with pytest.raises(rb.RbwsError) as e:
        rb.solve([P], mus, rb.default_opts(init=rb.INIT_LEARNED), bases=[basis])
    assert e.value.code == rb.ESTATE
