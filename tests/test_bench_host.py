"""Host-side logic of bench.py: the sweep's size set, the refusal of multi-GPU runs,
and the CPU baseline's record (run on a tiny sample, no GPU)."""
import json
import math
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _smooth357(n):
    for p in (3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def test_sweep_sizes_are_the_powers_of_two_and_the_3_5_7_smooth_sizes():
    s = bench.sweep_sizes()
    assert s == sorted(set(s))
    pow2 = [L for L in s if L & (L - 1) == 0]
    odd = [L for L in s if L & (L - 1)]
    assert pow2 == [1 << k for k in range(6, 23)]
    assert all(_smooth357(L) and 64 <= L <= 4e6 for L in odd)
    # every 3^a 5^b 7^c in [64, 4e6] is there (brute force over the exponents)
    want = {3 ** a * 5 ** b * 7 ** c for a in range(15) for b in range(10) for c in range(9)
            if 64 <= 3 ** a * 5 ** b * 7 ** c <= 4e6}
    assert set(odd) == want
    assert len(s) == 263 and len(pow2) == 17 and len(odd) == 246


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_cpu_baseline_record_on_a_tiny_sample(monkeypatch):
    # cpu_baseline pins OMP_NUM_THREADS for its workers: restored after the test
    monkeypatch.setenv("OMP_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", "0"))
    out = bench.cpu_baseline([64, 81, 125, 128, 243, 256], "c128", budget_s=5.0)
    assert out["kind"] == "oracle" and out["unit"] == "convs/s"
    host = out["host"]
    assert out["cores"] == host["threads"] >= 1 and host["nproc"] >= 1 and host["affinity"] >= 1
    assert out["cores"] <= host["affinity"]
    assert "sample" in out and "6 of 6" in out["sample"]
    assert math.isfinite(out["value"]) and out["value"] > 0


def test_roofline_is_the_compulsory_bytes_over_the_convolution_time(monkeypatch):
    """frac = (2L + M) b / (sum of the plan's launch durations per step) / 8 TB/s;
    traffic sums the counter bytes of every launch; the ratio is traffic / compulsory."""
    L, eb, steps = 1 << 22, 16, 4
    summ = {"col_fwd": {"launches": 8, "ms": 8 * 0.064, "mean_ms": 0.064, "mean_bytes": 2.0e8, "GBps": 3125.0},
            "row": {"launches": 4, "ms": 4 * 0.111, "mean_ms": 0.111, "mean_bytes": 4.0e8, "GBps": 3600.0},
            "col_bwd": {"launches": 4, "ms": 4 * 0.0756, "mean_ms": 0.0756, "mean_bytes": 2.7e8, "GBps": 3571.0}}
    counters = {"col_fwd": 2.0e8, "row": 4.0e8, "col_bwd": 2.7e8}
    monkeypatch.setattr(bench, "load_traffic", lambda k, w: counters[k])
    r = bench.roofline(summ, steps, L, eb, "tag", "col_fwd")
    conv_ms = 2 * 0.064 + 0.111 + 0.0756
    comp = (4 * L - 1) * eb
    assert r["algorithmic_bytes"] == comp
    assert abs(r["conv_ms"] - conv_ms) < 1e-9
    assert abs(r["achieved"] - comp / (conv_ms * 1e-3) / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert r["traffic"] == int(2 * 2.0e8 + 4.0e8 + 2.7e8)
    assert abs(r["traffic_ratio"] - r["traffic"] / comp) < 1e-3
    assert r["largest_kernel"]["kernel"] == "col_fwd" and r["all_kernels"]["col_fwd"]["launches_per_conv"] == 2
    monkeypatch.setattr(bench, "load_traffic", lambda k, w: None if k == "row" else 1.0)
    r = bench.roofline(summ, steps, L, eb, "tag", "col_fwd")
    assert r["traffic"] is None and r["traffic_ratio"] is None


def test_tuner_regret_against_the_exhaustive_table():
    """With a synthetic cost model, A1 choices equal to the exhaustive argmin have regret
    0 and a worse choice has exactly T(choice) / T(best) - 1."""
    def cost(L, M, m, D, dtype):  # known argmin: the m nearest 2L, all residues
        q = -(-M // m)
        return 1.0 + abs(math.log2(m) - math.log2(2 * L)) + (0.5 if D < q else 0.0)
    sizes = bench.sweep_sizes()
    from paper_2306_10016_amd import tune
    best = {}
    for L in sizes:
        t = tune.Tuner1D(tune.TuneDB(None), timer=cost).a0(L, 2 * L - 1, "c128")
        best[L] = t.params
    params = [dict(best[L]) for L in sizes]
    out = bench.tuner_regret(sizes, params, "c128", lambda *a: None, timer=cost)
    assert len(out["sizes"]) == 6 and out["worst_regret"] == 0.0
    i = sizes.index(out["sizes"][-1]["L"])
    params[i] = {"m": params[i]["m"] // 4, "D": 1}
    out = bench.tuner_regret(sizes, params, "c128", lambda *a: None, timer=cost)
    L = sizes[i]
    M = 2 * L - 1
    want = cost(L, M, params[i]["m"], 1, "c128") / min(
        cost(L, M, c["m"], c["D"], "c128") for c in tune.a0_candidates(L, M, "c128")) - 1
    assert out["sizes"][-1]["regret"] == pytest.approx(want, abs=1e-4)
    assert out["worst_regret"] > 0


def test_predictor_summary_reads_the_committed_evaluation():
    out = bench.predictor_summary()
    assert out is not None and "predictor_eval.json" in out["source"]
    assert out["checkpoint"] == "paper_2306_10016_amd/data/predictor.bin"
    assert os.path.exists(os.path.join(ROOT, out["checkpoint"]))
    assert len(out["heldout"]) >= 6 and all({"network", "default"} <= set(e) for e in out["heldout"])
