"""Writes blocks4_64_greedy.json: the oracle's greedy reduced basis at the
blocks4-64 workload's full size (64^3, four blocks, 512 seeded training
parameters, N = 30, Jacobi-PCG snapshots to 1e-12; Alg. 4 skeleton with the
residual-norm indicator), stored as digests so the GPU test can compare the
GPU build with it bit for bit without re-running the oracle (about 15 minutes
on 8 cores).

    python tests/golden/make_blocks4_64_greedy.py [--threads 8]

Calls only oracle/ and the seeded parameter generator.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2311_13862_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "blocks4_64_greedy.json")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    a = ap.parse_args()
    wl = W.blocks4_64()
    mut = W.sample_mu(wl.problem, wl.mu_lo, wl.mu_hi, wl.n_train, W.SEED_TRAIN)
    O = oracle.Problem(wl.problem)
    t = time.time()
    ob = oracle.greedy(O, mut, wl.N, wl.snap_tol, prec=oracle.PREC_JACOBI, nthreads=a.threads)
    el = time.time() - t
    N = ob.N
    steps = []
    for k in range(N):
        h = ob.hist[k]
        srt = np.sort(h)[::-1]
        steps.append({"selected": int(ob.selected[k]),
                      "hist_sha256": sha(h),
                      "hist_max": float(h.max()).hex(),
                      "hist_margin": float(srt[0] - srt[1]),
                      "v_sha256": sha(ob.V[k]),
                      "v_head": [float(v).hex() for v in ob.V[k][:4]]})
    doc = {"workload": wl.name, "n": wl.problem.n, "n_train": wl.n_train, "N": wl.N, "N_reached": N,
           "snap_tol": wl.snap_tol, "precond": "jacobi", "seed_train": W.SEED_TRAIN,
           "selected": [int(s) for s in ob.selected],
           "AqN_sha256": sha(ob.AqN[:, :N, :N]), "fN_sha256": sha(ob.fN[:N]),
           "steps": steps, "oracle_seconds": round(el, 1), "threads": a.threads}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {OUT}: N={N} in {el:.0f} s")


if __name__ == "__main__":
    main()
