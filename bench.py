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
    ap.add_argument("--reps", type=int, default=3,
                    help="interleaved repetitions of every start (zero, RB, learned, L1ROC) after the timed steps")
    ap.add_argument("--no-c2", action="store_true", help="skip the blocks4-64 FP64 leg")
    ap.add_argument("--spmv-only", action="store_true",
                    help="only the SpMV measurement (no autotuner launches: for profiling k_spmv)")
    ap.add_argument("--no-c5", action="store_true", help="skip the anisotropic mixed-size leg")
    ap.add_argument("--c5-ntrain", type=int, default=1024)
    ap.add_argument("--c5-batch", type=int, default=512)
    ap.add_argument("--c5-N", type=int, default=60)
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
    if args.spmv_only:
        spmv, by_tz, _, nb = spmv_leg(rbws, torch, P, mu, P.ndof, autotune=False)
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        rbws.stream_copy(a, b)  # calibrates a profiler's byte counters: each byte read and written once
        torch.cuda.synchronize()
        print(json.dumps({"spmv_only": True, "spmv_gbs": spmv, "copy_bytes": a.numel() * 8,
                          "spmv_gbs_by_tile_depth": {k: {str(t): v for t, v in d.items()} for k, d in by_tz.items()},
                          "spmv_batch": nb, "dispatch_order": "fp32 then fp64; tile depth 8, 16, 32; "
                          "per depth 1 untimed + 10 timed launches"}), flush=True)
        return

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
        rbws.stream_copy(a, b)  # the library's streaming copy: each byte read and written once
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "copy_bytes_read": a.numel() * 8,
                          "copy_bytes_written": b.numel() * 8,
                          "up2_sweep_algorithmic_bytes": float(np.sum(it * 20 - ou * 4)) * P.ndof,
                          "ap_sweep_algorithmic_bytes": float(np.sum(it * 12 - ou * 4)) * P.ndof,
                          "mg_pre0_algorithmic_bytes": vc * mg_pre0_bytes(spec.n) * P.ndof,
                          "mg_post0_algorithmic_bytes": vc * mg_post0_bytes(spec.n) * P.ndof,
                          "resid_pass_algorithmic_bytes": float(np.sum(12 + 24 * ou)) * P.ndof,
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

    # copy bandwidth of the device: the library's streaming copy kernel (16-byte
    # non-temporal loads and stores) and torch's copy, 1 GiB each way
    copy = copy_ceiling(rbws, torch)
    copy_gbs = copy["stream_copy"]

    # roofline of the dominant kernel (the single kernel with the most time over the timed
    # steps, from its HIP events), priced at its algorithmic bytes
    nd = P.ndof
    vcyc = np.array([s["vcycles"] for s in stats])
    alg = {"up2_sweep": args.steps * float(np.sum(iters * 20 - outer * 4)) * nd,  # R p, d, r; W d, r (FP32)
           "ap_sweep": args.steps * float(np.sum(iters * 12 - outer * 4)) * nd,   # R s, p_old; W p_new
           # V-cycle, finest level (FP32): R b, W x-sums of t; and R r, R ezy, W s
           "mg_pre0": args.steps * float(np.sum(vcyc)) * mg_pre0_bytes(spec.n) * nd,
           "mg_post0": args.steps * float(np.sum(vcyc)) * mg_post0_bytes(spec.n) * nd,
           # FP64 outer pass: the first R u, W b (12 B); each later one R u, d; W u', b (24 B)
           "resid_pass": args.steps * float(np.sum(12 + 24 * outer)) * nd}
    ms = {k: v[0] for k, v in kern.items()}
    n_launch = {k: v[1] for k, v in kern.items()}
    dom = max(alg, key=lambda k: ms.get(k, 0.0))
    dom_bytes = alg[dom]
    achieved = dom_bytes / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    per_launch_bytes = dom_bytes / max(n_launch[dom], 1)
    per_launch_ms = ms[dom] / max(n_launch[dom], 1)
    step_bytes = sum(alg.values()) / args.steps
    kern_frac = {k: round(alg[k] / (ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for k in alg if ms.get(k, 0) > 0}

    # set-up of the other starts: the paper's L1ROC basis and the learned start
    l1b = None
    l1_off = None
    if not args.no_l1roc:
        torch.cuda.synchronize()
        t = time.perf_counter()
        l1b = rbws.Basis.build(P, mu_train, args.N, wl.snap_tol, precond=rbws.PREC_JACOBI, method="l1roc")
        torch.cuda.synchronize()
        l1_off = time.perf_counter() - t
    net, learned_info = (None, None) if args.no_learned else train_learned(rbws, torch, W, wl, spec, basis, mu, args)

    # every start with the same preconditioner, precision, tolerance, kernel timer and
    # launch mode, interleaved in one process: zero, RB, learned, L1ROC, zero, RB, ...
    base = dict(precision=rbws.FP32_IR, tol=wl.tol, precond=PRECOND, eta_inner=args.eta,
                ir_mode=rbws.IR_RELIABLE, mg_omega=args.mg_omega, lift=rbws.LIFT_MFMA)
    legs = {}
    if not args.no_zero:
        zo = rbws.default_opts(init=rbws.INIT_ZERO, **base)
        legs["zero"] = lambda: rbws.solve([P], mu, zo)
    legs["rb"] = lambda: rbws.solve([P], mu, opts, bases=[basis])
    if net is not None:
        lo = rbws.default_opts(init=rbws.INIT_LEARNED, fallback=0, **base)
        legs["learned"] = lambda: rbws.solve([P], mu, lo, bases=[basis], mlps=[net])
    if l1b is not None:
        legs["l1roc"] = lambda: rbws.solve([P], mu, opts, bases=[l1b])
    cmp_runs = interleave(rbws, torch, legs, args.reps)
    starts = {k: leg_summary(rbws, v, args.batch) for k, v in cmp_runs.items()}
    if "zero" in cmp_runs:
        starts["rb"]["over_zero"] = paired_ratio(cmp_runs["rb"], cmp_runs["zero"])
    if "learned" in starts:
        st = cmp_runs["learned"]["stats"]
        starts["learned"].update(learned_info)
        starts["learned"]["started_from_mlp"] = int(np.sum(st["init_used"] == rbws.INIT_LEARNED))
        starts["learned"]["over_rb"] = paired_ratio(cmp_runs["learned"], cmp_runs["rb"])
        starts["learned"]["inner_iters_minus_rb"] = round(
            starts["learned"]["inner_iters_mean"] - starts["rb"]["inner_iters_mean"], 4)
        if "zero" in cmp_runs:
            starts["learned"]["over_zero"] = paired_ratio(cmp_runs["learned"], cmp_runs["zero"])
    if "l1roc" in starts:
        info = l1b.l1roc_info()
        starts["l1roc"].update({"rb_dim": l1b.N, "collocation_points": int(len(info["pts"])),
                                "t_off_s": round(l1_off, 2)})
    log(f"starts: { {k: v['value_median'] for k, v in starts.items()} }")

    c2 = None if args.no_c2 else c2_leg(rbws, torch, W, args)
    if c2 is not None:
        log(f"blocks4-64 FP64: {c2}")
    c5 = None if args.no_c5 else c5_leg(rbws, torch, W, args)
    if c5 is not None:
        log(f"aniso-mixed: {c5}")

    spmv, spmv_by_tz, spmv_tz, nb = spmv_leg(rbws, torch, P, mu, nd)
    log(f"SpMV GB/s: {spmv_by_tz}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(spec, mu, args.cpu_seconds, args.mg_omega, wl.tol)
        log(f"cpu baseline: {cpu}")

    zero = starts.get("zero")
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
        "zero_start_value": None if zero is None else zero["value_median"],
        "zero_start_inner_iters_mean": None if zero is None else zero["inner_iters_mean"],
        "rb_over_zero": None if zero is None else starts["rb"]["over_zero"]["median"],
        "starts": starts,
        "starts_protocol": (f"after the timed steps, every start once untimed, then {args.reps} rounds of "
                            f"{', '.join(starts)} in turn, same options, kernel timer on for all; "
                            "value_* from each run's wall time, over_* the median and range of the ratios "
                            "of runs in the same round"),
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_note": "completion time of each solve inside its batch (device clock), RB start",
        "t_off_s": round(t_off, 2),
        "bep": break_even(t_off, starts),
        "blocks4_64_fp64": c2,
        "aniso_mixed": c5,
        "spmv_gbs": {k: round(v, 1) for k, v in spmv.items()},
        "spmv_gbs_by_tile_depth": {k: {str(t): v for t, v in d.items()} for k, d in spmv_by_tz.items()},
        "spmv_batch": nb,
        "tile_depth": {"solve": tz, "spmv": spmv_tz, "solve_candidates_ms": {str(k): round(v, 3) for k, v in tz_ms.items()},
                       "picked_by": "short solves of half the batch at each depth"},
        "kernel_ms": {k: round(v, 2) for k, v in ms.items()},
        "kernel_launches": n_launch,
        "launches_before_timed_step": {k: v[1] for k, v in pre.items()},
        "kernel_frac_of_peak": kern_frac,
        "step_frac_of_peak": round(step_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_gbs": copy,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_per_launch(dom), "bytes_per_launch": per_launch_bytes,
                     "ms_per_launch": per_launch_ms, "frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def spmv_leg(rbws, torch, P, mu, nd, autotune=True):
    """SpMV bandwidth: 256 solves at 128^3 (2.1 GB per FP32 vector, far beyond the
    256 MB last-level cache); smaller batches leave the last round of workgroups
    part-empty.  The library's autotuner picks a depth from short runs on a zero
    vector; the bench also times 10 launches on random data at depths 8, 16 and 32
    and reports the fastest (every depth computes the same y).  Per precision and
    depth: one untimed launch, then the 10 timed ones."""
    spmv, spmv_by_tz = {}, {}
    nb = 256
    rbws.set_tuning(rbws.TUNE_TZ, 0)
    spmv_tz = rbws.autotune(P, nb, rbws.FP32_IR)[0] if autotune else None
    for name, dt, bpd, prec in (("fp32", torch.float32, 8, rbws.FP32_IR), ("fp64", torch.float64, 16, rbws.FP64)):
        x = torch.randn(nb, nd, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        spmv_by_tz[name] = {}
        for tzs in (8, 16, 32):
            rbws.set_tuning(rbws.TUNE_TZ, tzs)
            P.spmv(mu[:nb], x, y, precision=prec)
            rbws.profile(True, reset=True)
            for _ in range(10):
                P.spmv(mu[:nb], x, y, precision=prec)
            torch.cuda.synchronize()
            kk = rbws.profile(False, reset=True)["spmv"]
            spmv_by_tz[name][tzs] = round(bpd * nb * nd / (kk[0] / kk[1] * 1e-3) / 1e9, 1)
        spmv[name] = max(spmv_by_tz[name].values())
        del x, y
    rbws.set_tuning(rbws.TUNE_TZ, 0)
    return spmv, spmv_by_tz, spmv_tz, nb


def copy_ceiling(rbws, torch, reps=10):
    """GB/s (bytes read + written) of a 1 GiB device-to-device copy: the library's
    streaming copy kernel and torch's copy_, each timed with HIP events on the
    current stream, on which both are launched."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("stream_copy", lambda: rbws.stream_copy(a, b)), ("torch_copy", lambda: b.copy_(a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(reps * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    assert bool(torch.equal(a, b))
    del a, b
    return out


def interleave(rbws, torch, legs, reps):
    """Each leg once untimed (set-up), then `reps` rounds that run every leg once
    in turn.  Every run has the kernel timer on (the same launch mode for all).
    Returns per leg the wall seconds of each run, the last run's statistics and
    the kernel times summed over the timed runs."""
    for f in legs.values():
        f()
    out = {k: {"s": [], "stats": None, "kern": {}} for k in legs}
    for _ in range(reps):
        for k, f in legs.items():
            rbws.profile(True, reset=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = f()
            torch.cuda.synchronize()
            out[k]["s"].append(time.perf_counter() - t)
            out[k]["stats"] = st
            for kk, (m, n) in rbws.profile(False, reset=True).items():
                a = out[k]["kern"].setdefault(kk, [0.0, 0])
                a[0] += m
                a[1] += n
    return out


def leg_summary(rbws, run, batch):
    v = batch / np.array(run["s"])
    st = run["stats"]
    nrun = len(run["s"])
    stage = {k: round(run["kern"][k][0] / nrun, 3) for k in ("rb_project", "rb_coeffs", "lift_mfma")
             if run["kern"].get(k, (0.0, 0))[1] > 0}
    return {"value_median": round(float(np.median(v)), 3), "value_min": round(float(v.min()), 3),
            "start_stage_ms": stage,
            "value_max": round(float(v.max()), 3), "runs": [round(float(x), 3) for x in v],
            "all_converged": bool(np.all(st["status"] == rbws.SOLVE_CONVERGED)),
            "inner_iters_mean": float(np.mean(st["iters"])), "outer_iters_mean": float(np.mean(st["outer_iters"])),
            "init_relres_median": float(np.median(np.sqrt(st["init_rr"] / st["ff"]))),
            "max_final_relres": float(np.max(np.sqrt(st["final_rr"] / st["ff"])))}


def paired_ratio(a, b):
    """Throughput ratio a/b of the runs of the same round."""
    r = np.array(b["s"]) / np.array(a["s"])
    return {"median": round(float(np.median(r)), 4), "min": round(float(r.min()), 4), "max": round(float(r.max()), 4)}


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


def train_learned(rbws, torch, W, wl, spec, basis, mu, args):
    """Learned start: (mu, c(mu)) pairs from the reduced solve, a perceptron
    trained on the GPU on them, and its coefficient error against the reduced
    solve on the test batch."""
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
    return net, {"coef_relerr_vs_rb_median": float(np.median(cerr)), "train_pairs": args.mlp_pairs,
                 "train_epochs": args.mlp_epochs, "t_pairs_s": round(t_pairs, 3), "t_train_s": round(t_train, 3),
                 "final_loss": float(np.mean(hist[-32:])), "fallback": "strict (smaller true residual of u_MLP, u_RB)",
                 "network": f"{spec.p}-256-256-256-{basis.N} GELU, BF16 MFMA / FP32 Adam"}


def c2_leg(rbws, torch, W, args):
    """blocks4-64: the plain method in FP64 on the GPU.  Four blocks at 64^3,
    greedy basis N = 30 from 512 training parameters, 256 test parameters in
    one batched solve to relative residual 1e-10 by Jacobi-PCG (Alg. 1) from
    the RB start (Alg. 5) and from zero, interleaved.  The FP64 sweeps' roofline
    is priced at 24 (A p sweep, 16 on a restart) and 40 (update sweep) bytes per
    unknown and iteration, and 16 per residual evaluation."""
    wl = W.blocks4_64()
    spec = wl.problem
    P = rbws.Problem(spec)
    mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    mu = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, wl.n_test, W.SEED_TEST)
    rbws.set_tuning(rbws.TUNE_TZ, 0)  # the library's default tile depth for this size
    torch.cuda.synchronize()
    t = time.perf_counter()
    basis = rbws.Basis.build(P, mut, wl.N, wl.snap_tol, precond=rbws.PREC_JACOBI)
    torch.cuda.synchronize()
    t_off = time.perf_counter() - t
    base = dict(precision=rbws.FP64, tol=wl.tol, precond=rbws.PREC_JACOBI, lift=rbws.LIFT_MFMA)
    zo = rbws.default_opts(init=rbws.INIT_ZERO, **base)
    ro = rbws.default_opts(init=rbws.INIT_RB, **base)
    runs = interleave(rbws, torch, {"zero": lambda: rbws.solve([P], mu, zo),
                                    "rb": lambda: rbws.solve([P], mu, ro, bases=[basis])}, args.reps)
    out = {k: leg_summary(rbws, v, len(mu)) for k, v in runs.items()}
    out["rb"]["over_zero"] = paired_ratio(runs["rb"], runs["zero"])
    nd = P.ndof
    roof = {}
    for k, run in runs.items():
        st = run["stats"]
        it, ex = st["iters"].astype(np.int64), st["extra_spmv"].astype(np.int64)
        restarts = np.where(it > 0, np.maximum(ex, 1), 0)
        alg = {"ap_sweep": float(np.sum(24 * it - 8 * restarts)) * nd * args.reps,
               "up2_sweep": float(np.sum(40 * it)) * nd * args.reps,
               "resid_pass": float(np.sum(16 * (1 + ex))) * nd * args.reps}
        r = {}
        for kk, b in alg.items():
            ms, nl = run["kern"].get(kk, (0.0, 0))
            if ms > 0:
                gbs = b / (ms * 1e-3) / 1e9
                r[kk] = {"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "ms_per_launch": round(ms / max(nl, 1), 4), "bytes_per_launch": b / max(nl, 1)}
        roof[k] = r
    tz = {k: v for k, v in roof["rb"].items() if k != "resid_pass"}
    dom = max(tz, key=lambda k: runs["rb"]["kern"][k][0]) if tz else None
    return {"config": {"workload": "blocks4-64^3-fp64", "n": spec.n, "batch": len(mu), "rb_dim": basis.N,
                       "n_train": wl.n_train, "tol": wl.tol, "precond": "jacobi", "dtype": "f64",
                       "snap_tol": wl.snap_tol},
            "value": out["rb"]["value_median"], "unit": "mu-solves/s", "zero": out["zero"], "rb": out["rb"],
            "t_off_s": round(t_off, 2), "bep": break_even(t_off, out),
            "roofline": {"bound": "hbm", "kernel": dom, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         **({} if dom is None else roof["rb"][dom])},
            "sweeps": roof}


C5_SIZES = (64, 96, 128)


def c5_leg(rbws, torch, W, args):
    """aniso-mixed: 512 solves (solve i on grid C5_SIZES[i mod 3]) of the
    anisotropic octant problem with the Gaussian source (27 parameters) in one
    launch; per-size greedy bases (N = 60) and perceptrons (27-256-256-256-60);
    FP32 PCG with the V-cycle inside FP64 refinement to 1e-10, from zero, RB and
    learned starts, interleaved.  Per-solve latency is each solve's completion
    time inside the uneven batch (device clock)."""
    probs, bases, nets, specs, info, l1bases = [], [], [], [], [], []
    rbws.set_tuning(rbws.TUNE_TZ, 0)
    t_off = 0.0
    t_learn = 0.0
    for q, n in enumerate(C5_SIZES):
        wl = W.aniso_mixed(n)
        spec = wl.problem
        P = rbws.Problem(spec)
        mut = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, args.c5_ntrain, W.SEED_TRAIN + 10 * q)
        torch.cuda.synchronize()
        t = time.perf_counter()
        B = rbws.Basis.build(P, mut, args.c5_N, wl.snap_tol, precond=rbws.PREC_JACOBI)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t
        t_off += tb
        torch.cuda.synchronize()
        t = time.perf_counter()
        L1 = rbws.Basis.build(P, mut, min(args.c5_N, 60), wl.snap_tol, precond=rbws.PREC_JACOBI, method="l1roc")
        torch.cuda.synchronize()
        tl1 = time.perf_counter() - t
        l1bases.append(L1)
        mup = W.sample_mu(spec, wl.mu_lo, wl.mu_hi, args.mlp_pairs, W.SEED_MLP_PAIRS + 10 * q)
        t = time.perf_counter()
        c = B.coeffs(mup)
        net = rbws.Mlp.create(spec.p, B.N, hidden=256, depth=3, log_cols=24, in_m=0.0, in_s=1.0,
                              lin_lo=0.25, lin_hi=0.75, out_pow=1.0, seed=W.SEED_MLP_INIT + 10 * q)
        net.fit_output_scaling(mup, c)
        hist = net.train(mup, c, epochs=args.mlp_epochs, batch=256, lr=1e-3, lr_min=1e-5,
                         seed=W.SEED_MLP_PAIRS + 10 * q)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t
        t_learn += tl
        probs.append(P)
        bases.append(B)
        nets.append(net)
        specs.append(spec)
        info.append({"n": n, "rb_dim": B.N, "t_off_s": round(tb, 2), "t_learn_s": round(tl, 2),
                     "final_max_indicator": B.final_max, "final_loss": float(np.mean(hist[-32:])),
                     "l1roc_dim": L1.N, "l1roc_points": int(len(L1.l1roc_info()["pts"])),
                     "l1roc_t_off_s": round(tl1, 2)})
        log(f"aniso-mixed {n}^3: basis N={B.N} in {tb:.1f} s, L1ROC N={L1.N} in {tl1:.1f} s, "
            f"network in {tl:.1f} s")
    nsol = args.c5_batch
    assign = (np.arange(nsol) % 3).astype(np.int32)
    mu = np.empty((nsol, specs[0].p))
    for q in range(3):
        cnt = int(np.sum(assign == q))
        mu[assign == q] = W.sample_mu(specs[q], 0.1, 10.0, cnt, W.SEED_TEST + 10 * q)
    base = dict(precision=rbws.FP32_IR, tol=1e-10, precond=PRECOND, eta_inner=args.eta,
                ir_mode=rbws.IR_RELIABLE, mg_omega=args.mg_omega, lift=rbws.LIFT_MFMA)
    legs = {"zero": lambda: rbws.solve(probs, mu, rbws.default_opts(init=rbws.INIT_ZERO, **base), problem_of=assign),
            "rb": lambda: rbws.solve(probs, mu, rbws.default_opts(init=rbws.INIT_RB, **base), problem_of=assign,
                                     bases=bases),
            "learned": lambda: rbws.solve(probs, mu, rbws.default_opts(init=rbws.INIT_LEARNED, fallback=0, **base),
                                          problem_of=assign, bases=bases, mlps=nets),
            "l1roc": lambda: rbws.solve(probs, mu, rbws.default_opts(init=rbws.INIT_RB, **base), problem_of=assign,
                                        bases=l1bases)}
    runs = interleave(rbws, torch, legs, args.reps)
    out = {}
    for k, run in runs.items():
        sm = leg_summary(rbws, run, nsol)
        st = run["stats"]
        lat = st["t_done_ms"]
        sm["latency_ms_p50"] = round(float(np.percentile(lat, 50)), 3)
        sm["latency_ms_p99"] = round(float(np.percentile(lat, 99)), 3)
        sm["inner_iters_by_size"] = {str(n): float(np.mean(st["iters"][assign == q])) for q, n in enumerate(C5_SIZES)}
        if k == "learned":
            sm["started_from_mlp"] = int(np.sum(st["init_used"] == rbws.INIT_LEARNED))
        out[k] = sm
    out["rb"]["over_zero"] = paired_ratio(runs["rb"], runs["zero"])
    out["learned"]["over_rb"] = paired_ratio(runs["learned"], runs["rb"])
    out["learned"]["over_zero"] = paired_ratio(runs["learned"], runs["zero"])
    out["l1roc"]["over_zero"] = paired_ratio(runs["l1roc"], runs["zero"])
    return {"config": {"workload": "aniso27-mixed-64/96/128^3-fp32ir", "sizes": list(C5_SIZES), "batch": nsol,
                       "assignment": "solve i on size index i mod 3", "rb_dim": args.c5_N, "n_train": args.c5_ntrain,
                       "tol": 1e-10, "precond": "mg-vcycle" if PRECOND == 2 else "jacobi", "p": specs[0].p,
                       "mlp_pairs": args.mlp_pairs, "mlp_epochs": args.mlp_epochs},
            "value": out["rb"]["value_median"], "unit": "mu-solves/s", "per_size": info,
            "t_off_s": round(t_off, 2), "t_learn_s": round(t_learn, 2),
            "zero": out["zero"], "rb": out["rb"], "learned": out["learned"], "l1roc": out["l1roc"],
            "online_stage_note": ("start_stage_ms per batch: rb_project = V^T f(mu) on the matrix cores (Galerkin), "
                                  "rb_coeffs = reduced solves (Galerkin: assembly + Cholesky; L1ROC: the source at "
                                  "its collocation points + QR), lift_mfma = u0 = V c")}


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


def break_even(t_off, starts):
    """The paper's break-even point (Sec. 4.1): BEP = t_off / (t_on(MGCG) -
    t_on(RBWS)), the number of online solves after which the offline stage has
    paid for itself.  t_on is the mean online time per solve, here the inverse
    median batched throughput; the zero start with the same preconditioner
    plays MGCG.  For the learned start t_off also counts the training pairs and
    training, for L1ROC its own build.  None where a start is not faster than
    the zero start."""
    if "zero" not in starts:
        return None
    t_zero = 1.0 / starts["zero"]["value_median"]

    def bep(toff, v):
        gain = t_zero - 1.0 / v
        return round(toff / gain, 1) if gain > 0 else None

    out = {"definition": "t_off / (t_on(zero start) - t_on(start)), t_on = 1 / median throughput",
           "t_on_ms": {k: round(1e3 / v["value_median"], 5) for k, v in starts.items()}}
    for k, v in starts.items():
        if k == "zero":
            continue
        toff = t_off
        if k == "learned":
            toff = t_off + v.get("t_pairs_s", 0.0) + v.get("t_train_s", 0.0)
            out["t_off_learned_s"] = round(toff, 3)
        elif k == "l1roc":
            toff = v.get("t_off_s", t_off)
        out[k] = bep(toff, v["value_median"])
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(spec, mu, budget_s, omega, tol):
    """The oracle's own solver for the same problem on the host cores, measured
    to convergence: `cores` parameters of the batch, one per thread, each solved
    by FP64 MGCG (the V-cycle of Alg. 2 in Alg. 1, the same levels, smoother and
    weight as the GPU's) from zero to relative residual `tol`.  The oracle has
    no reduced basis at this size (its greedy would take hours), so the start
    is zero.  Timed twice: with the oracle's correctly rounded inner products,
    and with plain FP64 loops in their place (a conventional CPU code); a
    variant whose first solve alone would exceed the budget is skipped."""
    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    O = oracle.Problem(spec)
    sample = mu[:cores]
    out = {"unit": "mu-solves/s", "cores": cores, "kind": "oracle", "cpu": cpu_model(),
           "host_cpus": os.cpu_count()}
    for name, naive in (("exact_dots", False), ("naive_dots", True)):
        oracle.core.set_naive_dots(naive)
        try:
            t = time.perf_counter()
            _, st = O.mgcg_batch(sample, tol=tol, omega=omega, maxit=400, nthreads=cores)
            wall = time.perf_counter() - t
        finally:
            oracle.core.set_naive_dots(False)
        its = [int(s["iters"]) for s in st]
        out[name] = {"value": round(cores / wall, 5), "wall_s": round(wall, 2),
                     "s_per_solve_one_core": round(wall, 3), "iters_mean": float(np.mean(its)),
                     "all_converged": all(int(s["status"]) == 0 for s in st)}
        if wall > budget_s:
            break
    out["value"] = out["exact_dots"]["value"]
    out["cpu_reference_throughput"] = out.get("naive_dots", {}).get("value")
    out["sample"] = (f"{cores} parameters of the batch, one per thread, FP64 MGCG from zero to {tol:g} "
                     "(each to its own convergence); value: correctly rounded dots, "
                     "cpu_reference_throughput: plain FP64 dot loops")
    return out


if __name__ == "__main__":
    main()
