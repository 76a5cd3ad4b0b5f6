#!/usr/bin/env python3
"""Benchmark of the reduced-basis warm-start solver on one MI355X.

Workload: the 3D diffusion problem on a 128^3 interior grid (2,097,152
unknowns) with a piecewise-constant coefficient on the 2x2x2 octant split
(8 parameters, log-uniform in [0.01, 100]); a greedy reduced basis of
dimension 40 from 1024 seeded training parameters; 1024 seeded test
parameters solved in one batch to relative residual 1e-10 with PCG in FP32
(preconditioned by the multigrid V-cycle of Alg. 2, i.e. MGCG; --precond
jacobi for Jacobi-PCG) inside FP64 iterative refinement, started from the RB
solution (the paper's Alg. 5) and, for comparison, from zero.

One step = the whole online path over the batch: reduced assembly and
Cholesky, MFMA lift u0 = V c, the refined Krylov solve.  The offline greedy
build is timed separately (t_off).  All inputs are synthetic and seeded.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `--counters` runs the offline build and one step, then
a plain 1 GiB copy, for rocprofv3 counter collection, and prints the
algorithmic bytes of that step instead.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
PRECOND = 2            # RBWS_PREC_MG


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--ntrain", type=int, default=1024)
    ap.add_argument("--N", type=int, default=40)
    ap.add_argument("--eta", type=float, default=0.05,
                    help="inner tolerance of the refinement (0.05: fewest outer passes without stragglers at 128^3)")
    ap.add_argument("--mg-omega", type=float, default=0.9,
                    help="Jacobi weight of the V-cycle's smoother (0.9: fewest iterations at 128^3)")
    ap.add_argument("--precond", choices=("mg", "jacobi"), default="mg",
                    help="P of Alg. 1: the multigrid V-cycle of Alg. 2 (default) or Jacobi")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-zero", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-l1roc", action="store_true")
    ap.add_argument("--mlp-pairs", type=int, default=8192)
    ap.add_argument("--mlp-epochs", type=int, default=200)
    ap.add_argument("--counters", action="store_true",
                    help="short run for rocprofv3 --pmc (a few refinement rounds)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve_step(rb, P, basis, mu, opts):
    return rb.solve([P], mu, opts, bases=[basis])


def main():
    args = parse()
    global PRECOND
    PRECOND = {"mg": 2, "jacobi": 1}[args.precond]
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(solves are independent per parameter: a batch splits across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_13862_amd import rbws
    from paper_2311_13862_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU visible"
    wl = W.octants_128()
    spec = wl.problem
    P = rbws.Problem(spec)
    mu_train = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, args.ntrain, W.SEED_TRAIN)
    mu = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, args.batch, W.SEED_TEST)

    log(f"offline: greedy N={args.N} from {args.ntrain} training parameters at {spec.n}^3")
    torch.cuda.synchronize()
    t = time.perf_counter()
    basis = rbws.Basis.build(P, mu_train, args.N, wl.snap_tol, precond=rbws.PREC_JACOBI)
    torch.cuda.synchronize()
    t_off = time.perf_counter() - t
    log(f"offline done in {t_off:.1f} s, N={basis.N}, max training indicator {basis.final_max:.3g}")

    opts = rbws.default_opts(precision=rbws.FP32_IR, tol=wl.tol, precond=PRECOND,
                             eta_inner=args.eta, init=rbws.INIT_RB, lift=rbws.LIFT_MFMA,
                             ir_mode=rbws.IR_RELIABLE, mg_omega=args.mg_omega)
    # launches are counted by kind from here on, so that a profiler's per-dispatch
    # records of the timed step can be told apart from those of the set-up below
    rbws.profile(True, reset=True)
    # tile depth for this grid size and batch (setup, like the offline stage)
    tz, tz_ms = pick_tile_depth(rbws, torch, P, mu, args)
    log(f"tile depth {tz}: {tz_ms}")
    if args.counters:
        # rocprofv3 counter run: one step as timed below, then a plain copy of known size
        pre = rbws.profile(True, reset=True)
        st = solve_step(rbws, P, basis, mu, opts)
        stp = rbws.profile(False, reset=True)
        it = np.array([s["iters"] for s in st])
        ou = np.array([s["outer_iters"] for s in st])
        vc = float(np.sum([s["vcycles"] for s in st]))
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "copy_bytes_read": a.numel() * 8,
                          "copy_bytes_written": b.numel() * 8,
                          "up2_algorithmic_bytes": float(np.sum(it * 20 - ou * 4)) * P.ndof,
                          "ap_algorithmic_bytes": float(np.sum(it * 12 - ou * 4)) * P.ndof,
                          "mg_pre0_algorithmic_bytes": vc * mg_pre0_bytes(spec.n) * P.ndof,
                          "mg_post0_algorithmic_bytes": vc * mg_post0_bytes(spec.n) * P.ndof,
                          "launches_before_step": {k: v[1] for k, v in pre.items()},
                          "launches_step": {k: v[1] for k, v in stp.items()},
                          "sources_sha256": kernel_sources_hash()}), flush=True)
        return

    for w in range(args.warmup):
        solve_step(rbws, P, basis, mu, opts)
        log(f"warmup step {w + 1} done")
    pre = rbws.profile(True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for k in range(args.steps):
        stats = solve_step(rbws, P, basis, mu, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = rbws.profile(False, reset=True)
    elapsed = t1 - t0
    value = args.steps * args.batch / elapsed
    log(f"timed {args.steps} step(s): {elapsed:.2f} s, {value:.2f} mu-solves/s")
    ok = all(s["status"] == rbws.SOLVE_CONVERGED for s in stats)
    iters = np.array([s["iters"] for s in stats])
    outer = np.array([s["outer_iters"] for s in stats])
    lat = np.array([s["t_done_ms"] for s in stats])
    relres = np.array([np.sqrt(s["final_rr"] / s["ff"]) for s in stats])

    # copy bandwidth of the device (a plain 1 GiB + 1 GiB copy), for context
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b

    # roofline of the dominant kernel (the single kernel with the most time over the timed
    # steps, from its HIP events), priced at its algorithmic bytes
    nd = P.ndof
    vcyc = np.array([s["vcycles"] for s in stats])
    alg = {"up2_sweep": args.steps * float(np.sum(iters * 20 - outer * 4)) * nd,  # R p, d, r; W d, r (FP32)
           "ap_sweep": args.steps * float(np.sum(iters * 12 - outer * 4)) * nd,   # R s, p_old; W p_new
           # V-cycle, finest level (FP32): R b, W x-sums of t; and R r, R ezy, W s
           "mg_pre0": args.steps * float(np.sum(vcyc)) * mg_pre0_bytes(spec.n) * nd,
           "mg_post0": args.steps * float(np.sum(vcyc)) * mg_post0_bytes(spec.n) * nd}
    ms = {k: v[0] for k, v in kern.items()}
    n_launch = {k: v[1] for k, v in kern.items()}
    dom = max(alg, key=lambda k: ms.get(k, 0.0))
    dom_bytes = alg[dom]
    achieved = dom_bytes / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    per_launch_bytes = dom_bytes / max(n_launch[dom], 1)
    per_launch_ms = ms[dom] / max(n_launch[dom], 1)

    # zero start with the same preconditioner, precision and tolerance
    zero_value = None
    zero_iters = None
    if not args.no_zero:
        zopts = rbws.default_opts(precision=rbws.FP32_IR, tol=wl.tol, precond=PRECOND,
                                  eta_inner=args.eta, init=rbws.INIT_ZERO, ir_mode=rbws.IR_RELIABLE,
                                  mg_omega=args.mg_omega)
        torch.cuda.synchronize()
        t = time.perf_counter()
        zst = rbws.solve([P], mu, zopts)
        torch.cuda.synchronize()
        zero_value = args.batch / (time.perf_counter() - t)
        zero_iters = float(np.mean([s["iters"] for s in zst]))
        log(f"zero start: {zero_value:.2f} mu-solves/s, mean inner iterations {zero_iters:.1f}")

    # the paper's own RB variant: an L1ROC basis from the same training set
    l1roc = None
    if not args.no_l1roc:
        l1roc = l1roc_leg(rbws, torch, wl, P, mu_train, mu, args)
        log(f"L1ROC start: {l1roc}")

    # learned start: a perceptron trained on the GPU on (mu, c(mu)) pairs of the reduced solve
    learned = None
    if not args.no_learned:
        learned = learned_leg(rbws, W, wl, spec, P, basis, mu, args)
        log(f"learned start: {learned}")

    # SpMV bandwidth: 256 solves at 128^3 (2.1 GB per FP32 vector, far beyond the 256 MB
    # last-level cache); smaller batches leave the last round of workgroups part-empty
    spmv = {}
    nb = 256
    rbws.set_tuning(rbws.TUNE_TZ, 0)  # the SpMV takes its own autotuned depth
    spmv_tz, _ = rbws.autotune(P, nb, rbws.FP32_IR)
    for name, dt, bpd, prec in (("fp32", torch.float32, 8, rbws.FP32_IR), ("fp64", torch.float64, 16, rbws.FP64)):
        x = torch.randn(nb, nd, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        P.spmv(mu[:nb], x, y, precision=prec)
        rbws.profile(True, reset=True)
        for _ in range(10):
            P.spmv(mu[:nb], x, y, precision=prec)
        torch.cuda.synchronize()
        kk = rbws.profile(False, reset=True)["spmv"]
        spmv[name] = bpd * nb * nd / (kk[0] / kk[1] * 1e-3) / 1e9
        del x, y
    log(f"SpMV GB/s: {spmv}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(spec, mu, float(np.mean(iters)), float(np.mean(outer)), args.cpu_seconds, args.mg_omega)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "mu-solves/s to rel-res 1e-10 @128^3 (RB warm start; zero start beside it)",
        "value": round(value, 3),
        "unit": "mu-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 outer",
        "data": "synthetic (seeded parameters)",
        "config": {"workload": "octants8-128^3-fp32ir-rbws", "n": spec.n, "batch": args.batch,
                   "rb_dim": basis.N, "n_train": args.ntrain, "tol": wl.tol, "precond": "mg-vcycle" if args.precond == "mg" else "jacobi",
                   "eta_inner": args.eta, "mg_omega": args.mg_omega, "refinement": "reliable-update", "init": "rb",
                   "lift": "mfma", "parallelism": "none"},
        "all_converged": bool(ok),
        "max_final_relres": float(relres.max()),
        "inner_iters_mean": float(iters.mean()),
        "outer_iters_mean": float(outer.mean()),
        "vcycles_mean": float(vcyc.mean()),
        "zero_start_value": None if zero_value is None else round(zero_value, 3),
        "zero_start_inner_iters_mean": zero_iters,
        "rb_over_zero": None if zero_value is None else round(value / zero_value, 4),
        "learned_start": learned,
        "l1roc_start": l1roc,
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "t_off_s": round(t_off, 2),
        "bep": break_even(t_off, value, zero_value, learned, l1roc),
        "spmv_gbs": {k: round(v, 1) for k, v in spmv.items()},
        "spmv_batch": nb,
        "tile_depth": {"solve": tz, "spmv": spmv_tz, "solve_candidates_ms": {str(k): round(v, 3) for k, v in tz_ms.items()},
                       "picked_by": "short solves of half the batch at each depth"},
        "kernel_ms": {k: round(v, 2) for k, v in ms.items()},
        "kernel_launches": n_launch,
        "launches_before_timed_step": {k: v[1] for k, v in pre.items()},
        "copy_gbs": round(copy_gbs, 1),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_per_launch(dom), "bytes_per_launch": per_launch_bytes,
                     "ms_per_launch": per_launch_ms, "frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def pick_tile_depth(rbws, torch, P, mu, args, cands=(16, 32, 64)):
    """Tile depth of the solve's sweeps and V-cycle kernels: a short solve
    (zero start, three outer steps) of half the batch at each candidate, timed;
    the fastest is kept for the rest of the run.  The library's own autotuner
    times a plain y = A x, whose best depth is shallower than the solve's."""
    sub = mu[: max(1, args.batch // 2)]
    o = rbws.default_opts(precision=rbws.FP32_IR, tol=1e-10, precond=PRECOND, eta_inner=args.eta,
                          init=rbws.INIT_ZERO, ir_mode=rbws.IR_RELIABLE, mg_omega=args.mg_omega, max_outer=3)
    ms = {}
    for tz in cands:
        rbws.set_tuning(rbws.TUNE_TZ, tz)
        rbws.solve([P], sub[:64], o)  # set-up for this depth
        torch.cuda.synchronize()
        t = time.perf_counter()
        rbws.solve([P], sub, o)
        torch.cuda.synchronize()
        ms[tz] = (time.perf_counter() - t) * 1e3
    best = min(ms, key=ms.get)
    rbws.set_tuning(rbws.TUNE_TZ, best)
    return best, ms


def learned_leg(rbws, W, wl, spec, P, basis, mu, args):
    """Pairs from the reduced solve, GPU training, then the batch from the learned
    start (strict fallback: per solve the smaller true residual of u_MLP, u_RB)."""
    import torch
    mup = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, args.mlp_pairs, W.SEED_MLP_PAIRS)
    torch.cuda.synchronize()
    t = time.perf_counter()
    c = basis.coeffs(mup)
    t_pairs = time.perf_counter() - t
    net = rbws.Mlp.create(spec.p, basis.N, hidden=256, depth=3, log_cols=spec.p, in_m=0.0, in_s=2.0,
                          out_pow=1.0, seed=W.SEED_MLP_INIT)
    net.fit_output_scaling(mup, c)
    t = time.perf_counter()
    hist = net.train(mup, c, epochs=args.mlp_epochs, batch=256, lr=1e-3, lr_min=1e-5, seed=W.SEED_MLP_PAIRS)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    c_rb = basis.coeffs(mu)
    c_nn = net.predict(mu)
    cerr = np.linalg.norm(c_nn - c_rb, axis=1) / np.linalg.norm(c_rb, axis=1)
    opts = rbws.default_opts(precision=rbws.FP32_IR, tol=wl.tol, precond=PRECOND,
                             eta_inner=args.eta, init=rbws.INIT_LEARNED, lift=rbws.LIFT_MFMA,
                             ir_mode=rbws.IR_RELIABLE, fallback=0, mg_omega=args.mg_omega)
    rbws.solve([P], mu[:64], opts, bases=[basis], mlps=[net])  # set-up of this start, like the others'
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = rbws.solve([P], mu, opts, bases=[basis], mlps=[net])
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    used = [s["init_used"] for s in st]
    return {"value": round(args.batch / el, 3), "unit": "mu-solves/s",
            "all_converged": all(s["status"] == rbws.SOLVE_CONVERGED for s in st),
            "inner_iters_mean": float(np.mean([s["iters"] for s in st])),
            "init_relres_median": float(np.median([np.sqrt(s["init_rr"] / s["ff"]) for s in st])),
            "started_from_mlp": int(sum(u == rbws.INIT_LEARNED for u in used)),
            "coef_relerr_vs_rb_median": float(np.median(cerr)),
            "train_pairs": args.mlp_pairs, "train_epochs": args.mlp_epochs, "t_pairs_s": round(t_pairs, 3),
            "t_train_s": round(t_train, 3), "final_loss": float(np.mean(hist[-32:])),
            "network": f"{spec.p}-256-256-256-{basis.N} GELU, BF16 MFMA / FP32 Adam"}


def mg_pre0_bytes(n):
    """Per finest-level point: read b (FP32) and write the restriction's x-sums
    of t = b - A e1 (n x n rows of nc = (n-1)//2 values per solve): the path
    for tiles that span whole rows (n <= 128)."""
    return 4.0 + 4.0 * ((n - 1) // 2) / n


def mg_post0_bytes(n):
    """Per finest-level point: read r, write s (FP32), and read the coarse
    correction (nc^3 values per solve, nc = (n-1)//2), which the kernel
    interpolates itself on tiles that span whole rows (n <= 128)."""
    nc = (n - 1) // 2
    return 8.0 + 4.0 * (nc / n) ** 3


KERNEL_SOURCES = ("fast.hpp", "ir.hip", "mg.hip", "stencil.hpp", "crdot.hpp", "rbws_internal.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fp32ir_mg_kernels_octants128_traffic.txt")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_13862_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's readings), or
    None when there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(l.split(":", 1) for l in fh if ":" in l and not l.startswith(("#", " ", "|")))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != kernel_sources_hash():
        return None
    v = kv.get(f"{kernel}_traffic_bytes_per_launch")
    return float(v) if v else None


def l1roc_leg(rbws, torch, wl, P, mu_train, mu, args):
    """The L1ROC start (Sec. 3.1, Alg. 4): greedy build on the training set
    (timed as its offline stage), then the batch refined from it exactly like
    the timed step (after one warm-up solve of the same batch)."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    lb = rbws.Basis.build(P, mu_train, args.N, wl.snap_tol, precond=rbws.PREC_JACOBI, method="l1roc")
    torch.cuda.synchronize()
    t_off = time.perf_counter() - t
    opts = rbws.default_opts(precision=rbws.FP32_IR, tol=wl.tol, precond=PRECOND, eta_inner=args.eta,
                             init=rbws.INIT_RB, lift=rbws.LIFT_MFMA, ir_mode=rbws.IR_RELIABLE,
                             mg_omega=args.mg_omega)
    rbws.solve([P], mu, opts, bases=[lb])
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = rbws.solve([P], mu, opts, bases=[lb])
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    info = lb.l1roc_info()
    return {"value": round(args.batch / el, 3), "unit": "mu-solves/s",
            "all_converged": bool(np.all(st["status"] == rbws.SOLVE_CONVERGED)),
            "inner_iters_mean": float(np.mean(st["iters"])), "outer_iters_mean": float(np.mean(st["outer_iters"])),
            "init_relres_median": float(np.median(np.sqrt(st["init_rr"] / st["ff"]))),
            "rb_dim": lb.N, "collocation_points": int(len(info["pts"])), "t_off_s": round(t_off, 2)}


def break_even(t_off, rb_value, zero_value, learned, l1roc=None):
    """The paper's break-even point (Sec. 4.1): BEP = t_off / (t_on(MGCG) -
    t_on(RBWS)), the number of online solves after which the offline stage has
    paid for itself.  t_on is the mean online time per solve, here the inverse
    batched throughput; the zero start with the same preconditioner plays MGCG.
    For the learned start t_off also counts the training pairs and training.
    None where a start is not faster than the zero start."""
    if zero_value is None:
        return None
    t_zero = 1.0 / zero_value

    def bep(toff, v):
        gain = t_zero - 1.0 / v
        return round(toff / gain, 1) if gain > 0 else None

    out = {"definition": "t_off / (t_on(zero start) - t_on(start)), t_on = 1 / throughput",
           "t_on_ms": {"zero": round(1e3 * t_zero, 5), "rb": round(1e3 / rb_value, 5)},
           "rb": bep(t_off, rb_value)}
    if learned is not None:
        toff_l = t_off + learned["t_pairs_s"] + learned["t_train_s"]
        out["t_on_ms"]["learned"] = round(1e3 / learned["value"], 5)
        out["learned"] = bep(toff_l, learned["value"])
        out["t_off_learned_s"] = round(toff_l, 3)
    if l1roc is not None:
        out["t_on_ms"]["l1roc"] = round(1e3 / l1roc["value"], 5)
        out["l1roc"] = bep(l1roc["t_off_s"], l1roc["value"])
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(spec, mu, gpu_inner_mean, gpu_outer_mean, budget_s, omega):
    """The oracle's own solver for the same method on the host cores, on a
    bounded sample: `cores` parameters in parallel (one per thread), each for a
    capped number of iterations; the per-solve cost is scaled to the GPU's mean
    inner iteration count.  With the multigrid preconditioner the oracle runs
    MGCG in FP64 (it has no FP32 inner solver for it), with Jacobi its FP32
    refinement solver."""
    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    O = oracle.Problem(spec)
    sample = mu[:cores]
    mg = PRECOND == 2

    def run(ms, cap, threads):
        if mg:
            O.mgcg_batch(ms, tol=1e-30, maxit=cap, nthreads=threads, omega=omega)
        else:
            O.ir_batch(ms, prec=oracle.PREC_JACOBI, tol=1e-10, eta=1e-30, kin_max=cap, max_outer=1,
                       nthreads=threads, reliable=True)

    # probe the cost of a few iterations, then size the sample to the budget
    t = time.perf_counter()
    run(sample[:1], 3, 1)
    per_it = max((time.perf_counter() - t) / 5.0, 1e-3)
    cap = int(max(3, min(400, budget_s / per_it / 2.0)))
    t = time.perf_counter()
    run(sample, cap, cores)
    wall = time.perf_counter() - t
    per_solve = wall / cap * (gpu_inner_mean + (0 if mg else 2 * gpu_outer_mean))
    what = "FP64 MGCG iterations" if mg else "FP32 inner iterations (+2 outer residuals)"
    return {"value": round(cores / per_solve, 5), "unit": "mu-solves/s", "cores": cores,
            "kind": "oracle", "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "s_per_solve_one_core": round(per_solve, 3),
            "sample": f"{cores} parameters of the batch, one per thread, {cap} {what} each; "
                      f"wall {wall:.1f} s, scaled to the GPU's mean {gpu_inner_mean:.0f} inner iterations per solve"}

if __name__ == "__main__":
    main()
