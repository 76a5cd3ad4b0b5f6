"""Host logic of bench.py (no GPU): the paper's break-even point, the
algorithmic bytes of the fused V-cycle kernels, and the one-GPU guard."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_break_even_point(bench):
    """BEP = t_off / (t_on(zero) - t_on(start)) with t_on = 1 / median throughput
    (Sec. 4.1); None where a start is not faster; the learned start's t_off adds
    pairs and training, L1ROC's is its own build."""
    starts = {"zero": {"value_median": 1000.0}, "rb": {"value_median": 1000.0 / 0.9},
              "learned": {"value_median": 1000.0 / 0.8, "t_pairs_s": 0.5, "t_train_s": 1.5},
              "l1roc": {"value_median": 900.0, "t_off_s": 2.0}}
    out = bench.break_even(6.0, starts)
    assert out["rb"] == pytest.approx(6.0 / (1e-3 - 0.9e-3), rel=1e-9)
    assert out["learned"] == pytest.approx(8.0 / (1e-3 - 0.8e-3), rel=1e-9)
    assert out["t_off_learned_s"] == pytest.approx(8.0)
    assert out["l1roc"] is None
    assert out["t_on_ms"]["zero"] == pytest.approx(1.0)
    assert bench.break_even(6.0, {"rb": {"value_median": 10.0}}) is None


def test_paired_ratio(bench):
    """Ratios of throughputs are taken between runs of the same round."""
    a = {"s": [1.0, 2.0, 4.0]}
    b = {"s": [2.0, 2.0, 2.0]}
    r = bench.paired_ratio(a, b)
    assert (r["median"], r["min"], r["max"]) == (1.0, 0.5, 2.0)


def test_algorithmic_bytes(bench):
    """Per finest-level point at 128^3 (n_c = 63): the pre-smoothing reads b and
    writes the x-sums (4 + 4 n_c / n), the post-smoothing reads r and the
    coarse correction and writes s (8 + 4 (n_c / n)^3)."""
    assert bench.mg_pre0_bytes(128) == pytest.approx(4.0 + 4.0 * 63 / 128)
    assert bench.mg_post0_bytes(128) == pytest.approx(8.0 + 4.0 * (63 / 128) ** 3)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""
