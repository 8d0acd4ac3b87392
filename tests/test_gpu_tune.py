"""The tuner and predictor entry points of include/hdc_tune.h on the GPU, called
through ctypes:

* hdc_tune (A0, section 4.2; A1, section 4.3) times every candidate on the
  device and appends it to the JSON-lines database; its choice is the argmin
  of its own rows under the tie rule, the Python reader of the same database
  agrees, and A1 then reuses it without timing.
* Plans built from tuner parameters (hdc_plan_params) with non-default column
  tiles give the default tile's result bit for bit, and the oracle's.
* hdc_predict evaluates a saved network in the HIP kernels and picks the same
  per-axis parameters as the Python predictor running the same network.
"""
import json

import numpy as np
import pytest

import oracle
from gpu_util import TOL, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")
from paper_2306_10016_amd import predict, tune  # noqa: E402


def _argmin(rows):
    """The tie rule of the tuner: within 1 % of the fastest, the smaller m, then D, then the default tile."""
    lo = min(ms for _, ms in rows)

    def key(p):
        m = p["m"] if isinstance(p["m"], list) else [p["m"]]
        D = p["D"] if isinstance(p["D"], list) else [p["D"]]
        t = p.get("tile", [0] * len(m))
        t = t if isinstance(t, list) else [t]
        return (m, D, [0 if x == 0 else 1 + x for x in t])
    near = [(p, ms) for p, ms in rows if ms <= lo * 1.01]
    return min(near, key=lambda r: (key(r[0]), r[1]))[0]


@pytest.mark.parametrize("L,M,dtype", [(3000, 5999, "c128"), (70000, 139999, "c64")])
def test_tune_a0_1d_is_the_argmin_of_its_database(tmp_path, L, M, dtype):
    path = str(tmp_path / "db.jsonl")
    say(f"hdc_tune A0 1D L={L} {dtype}")
    db = tune.TuneDB(path, device=tune.device_name(), build=tune.build_hash())
    r, best = tune.run_search(db, L, M, dtype, tune.A0)
    rows = r.table
    assert len(rows) >= 4
    for line in open(path):
        rec = json.loads(line)
        assert rec["device"] == tune.device_name() and rec["build"] == tune.build_hash()
    assert r.params == _argmin(rows)
    assert best.p[0] == -(-L // best.m[0]) and best.q[0] == -(-M // best.m[0])
    # A1 on the same database reuses the choice without timing (the Python reader agrees)
    again = tune.Tuner1D(tune.TuneDB(path, device=tune.device_name(), build=tune.build_hash())).a1(L, M, dtype)
    assert again.source == "db" and again.params == r.params
    # the chosen plan convolves correctly
    f, g, f64, g64 = inputs(L, 800, L % 97, dtype)
    h = to_host(hdc.Plan.from_params(L, M, dtype, r.params).convolve(to_dev(f), to_dev(g)))
    assert rel(h, oracle.padded_1d(f64, g64, M)) <= TOL[dtype]


def test_tune_a1_then_nd_a0(tmp_path):
    path = str(tmp_path / "db.jsonl")
    db = tune.TuneDB(path, device=tune.device_name(), build=tune.build_hash())
    say("hdc_tune A1 1D sequence")
    for L in (2000, 9000, 40000):
        r = tune.Tuner1D(db).a1(L, 2 * L - 1, "c128")
        assert r.source == "A1" and len(r.table) >= 2
        assert r.params == _argmin(r.table)
    say("hdc_tune A0 2D 300x200 c64")
    r, best = tune.run_search(db, [300, 200], [599, 399], "c64", tune.A0)
    assert len(r.params["m"]) == 2 and best.C[0] == 399 and best.C[1] == 1
    f, g, f64, g64 = inputs((300, 200), 801, 0, "c64")
    h = to_host(hdc.Plan.from_params([300, 200], [599, 399], "c64", r.params).convolve(to_dev(f), to_dev(g)))
    assert rel(h, oracle.padded_nd(f64, g64, (599, 399))) <= TOL["c64"]


# (L, M, m, dtype, tiles): column/row plans and an N-D outer axis, with the
# tiles half and double the default where the kernels allow them
TILE_CASES = [
    (100000, 199999, 1 << 17, "c128", [16, 128]),  # m1 = 32: default 64 columns
    (100000, 199999, 1 << 17, "c64", [32, 128]),   # default 64
    (600000, 1199999, 1 << 20, "c128", [4, 16]),   # m1 = 256: default 8
    (3000000, 5999999, 1 << 22, "c128", [4]),      # m1 = 1024: default 8
    (3000000, 5999999, 1 << 22, "c64", [4]),       # default 8
]


@pytest.mark.parametrize("L,M,m,dtype,tiles", TILE_CASES)
def test_column_tiles_give_the_same_result(L, M, m, dtype, tiles):
    say(f"tiles L={L} m={m} {dtype} {tiles}")
    f, g, f64, g64 = inputs(L, 802, L % 89, dtype)
    ft, gt = to_dev(f), to_dev(g)
    ref = to_host(hdc.Plan.from_params(L, M, dtype, {"m": m, "D": 0}).convolve(ft, gt))
    for t in tiles:
        h = to_host(hdc.Plan.from_params(L, M, dtype, {"m": m, "D": 0, "tile": t}).convolve(ft, gt))
        assert np.array_equal(h, ref), t
    if L <= 100000:
        assert rel(ref, oracle.padded_1d(f64, g64, M)) <= TOL[dtype]


def test_nd_outer_axis_tiles():
    say("tiles 2D 600x300 c64")
    Ls, Ms = [600, 300], [1199, 599]
    f, g, f64, g64 = inputs(tuple(Ls), 803, 0, "c64")
    ft, gt = to_dev(f), to_dev(g)
    ref = to_host(hdc.Plan.from_params(Ls, Ms, "c64", {"m": [1024, 512], "D": [0, 0]}).convolve(ft, gt))
    h = to_host(hdc.Plan.from_params(Ls, Ms, "c64", {"m": [1024, 512], "D": [0, 0], "tile": [4, 0]}).convolve(ft, gt))
    assert np.array_equal(h, ref)
    assert rel(ref, oracle.padded_nd(f64, g64, tuple(Ms))) <= TOL["c64"]


def test_predict_matches_the_python_predictor(tmp_path):
    """A saved network through hdc_predict (features, HIP forward, class mapping in the
    library) against the Python predictor running the same weights."""
    say("hdc_predict vs Python predictor")
    py = predict.Predictor(seed=5)
    path = str(tmp_path / "net.bin")
    py.save(path)
    cp = predict.CheckpointPredictor(path)
    probs = [([4096, 4096], "c64"), ([8192, 8192], "c64"), ([256, 256, 256], "c64"), ([100000], "c128"),
             ([1000, 37], "c128"), ([64, 3000, 5], "c64")]
    for Ls, dt in probs:
        Ms = [2 * L - 1 for L in Ls]
        want, wconf, _ = py.predict_axes(Ls, Ms, dt)
        got, gconf = cp.predict_axes(Ls, Ms, dt)
        assert got == [tuple(w) for w in want], (Ls, got, want)
        assert np.allclose(gconf, wconf, rtol=1e-5, atol=1e-6)
    cp.close()
