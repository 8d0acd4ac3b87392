"""Host logic of the autotuner (section 4) and of the predictor's encoding, run
against a deterministic synthetic cost model instead of GPU timings.  The
timings themselves are machine-dependent: parity unpinned for those; here the
searches are pinned to the known argmin of the synthetic model."""
import json
import math
import os

import numpy as np
import pytest

import paper_2306_10016_amd as hdc
from paper_2306_10016_amd import predict, tune


def cost_model(L, M, m, D, dtype):
    """A bowl in log2(m) with its minimum at m* = 2^ceil(log2 L) / 4, plus a penalty for D < q."""
    q = -(-M // m)
    mstar = tune.pow2_ceil(L) / 4
    return 1.0 + (math.log2(m) - math.log2(mstar)) ** 2 + (0.5 if D < q else 0.0)


@pytest.mark.parametrize("L", [37, 1000, 4096, 100000, 3 ** 13])
def test_candidates_are_admissible(L):
    """Every parameter set the library's A0 times is admissible (section 2.5) and in the
    class grid: p = ceil(L/m) in the classes or q = 1."""
    M = 2 * L - 1
    cands = tune.a0_candidates(L, M, "c64")
    assert cands
    for c in cands:
        m, D = c["m"], c["D"]
        d = hdc.derive(L, M, m, D=D, dtype="c64")
        assert d["p"] * m >= L and d["q"] * m >= M and d["q"] >= d["p"]
        assert m & (m - 1) == 0 or (d["variant"] == 0 and m <= 4096)  # m = R 2^k: the fused kernel
        assert d["p"] in tune.P_CLASSES or d["q"] == 1
        assert D == d["q"] or (D & (D - 1)) == 0  # all residues, or a power of two per pass
    grid = {(c["m"], c["D"]) for c in cands if "tile" not in c}
    assert len(grid) == len([c for c in cands if "tile" not in c])  # each timed once


def test_a0_finds_the_model_argmin():
    t = tune.Tuner1D(tune.TuneDB(None), timer=cost_model)
    r = t.a0(5000, 9999, "c64")
    assert r.params["m"] == tune.pow2_ceil(5000) // 4 and r.params["D"] == -(-9999 // r.params["m"])
    assert "tile" not in r.params  # the tiles cost the same: the default wins the tie
    assert r.source == "A0"


def test_a1_uses_experience_and_matches_a0_with_fewer_timings():
    calls = []

    def counting(L, M, m, D, dt):
        calls.append((L, m, D))
        return cost_model(L, M, m, D, dt)
    db = tune.TuneDB(None)
    t = tune.Tuner1D(db, timer=counting)
    for L in (2000, 4000, 8000):  # experience accumulates
        t.a1(L, 2 * L - 1, "c64")
    calls.clear()
    r = t.a1(16000, 31999, "c64")
    a0 = tune.Tuner1D(tune.TuneDB(None), timer=cost_model).a0(16000, 31999, "c64")
    assert r.params == a0.params
    assert r.source == "A1"
    assert len(calls) < len(tune.a0_candidates(16000, 31999, "c64"))


def test_db_reuse_and_resume(tmp_path):
    path = str(tmp_path / "db.jsonl")
    t = tune.Tuner1D(tune.TuneDB(path, device="dev", build="b1"), timer=cost_model)
    r1 = t.a1(3000, 5999, "c128")
    # a run killed mid-line leaves a partial record: the reader skips it
    with open(path, "a") as fh:
        fh.write('{"key": "trunc')
    db2 = tune.TuneDB(path, device="dev", build="b1")
    r2 = tune.Tuner1D(db2, timer=lambda *a: pytest.fail("should not time")).a1(3000, 5999, "c128")
    assert r2.source == "db" and r2.params == r1.params
    # another build does not reuse the timings
    db3 = tune.TuneDB(path, device="dev", build="b2")
    assert db3.best(tune.problem_key(3000, 5999, "c128")) is None
    # a search after the cut line appends whole records that read back
    tune.Tuner1D(db3, timer=cost_model).a0(700, 1399, "c128")
    db4 = tune.TuneDB(path, device="dev", build="b2")
    assert db4.best(tune.problem_key(700, 1399, "c128")) is not None


def test_tie_rule_prefers_smaller_m_then_D():
    """Within 1 % of the fastest: the smaller m, then the smaller D."""
    table = {(64, 2): 1.000, (32, 4): 1.005, (32, 1): 1.009}

    def cost(L, M, m, D, dt):
        return table.get((m, D), 2.0)
    r = tune.Tuner1D(tune.TuneDB(None), timer=cost).a0(100, 199, "c128")
    assert r.params == {"m": 32, "D": 1}


def test_nd_a0_is_separable_per_axis():
    """N-D A0 searches each axis with the others at their defaults and returns the
    per-axis argmins combined (section 4.2)."""
    want = {0: 64, 1: 256}

    def cost(pr, pm):
        t = 1.0
        for a in range(2):
            t += abs(math.log2(pm.m[a]) - math.log2(want[a])) + (0.3 if pm.D[a] < pm.q[a] else 0.0)
        return t
    r, best = tune.run_search(tune.TuneDB(None), [200, 300], [399, 599], "c64", tune.A0, cost)
    assert r.params["m"] == [64, 256] and list(best.D[:2]) == list(best.q[:2])
    assert best.p[0] == 4 and best.p[1] == 2 and best.C[0] == 599 and best.C[1] == 1


def test_regret():
    assert tune.regret(1.1, 1.0) == pytest.approx(0.1)
    assert tune.regret(1.0, 1.0) == 0.0


@pytest.mark.parametrize("L", [64, 1000, 8192, 100000])
def test_predictor_classes_round_trip(L):
    M = 2 * L - 1
    seen = set()
    for ci, (pc, dm) in enumerate(predict.CLASSES):
        m, D = predict.params_of(ci, L, M, outer=False)
        q = -(-M // m)
        if ci == predict.EXPLICIT:  # explicit padding: one residue
            assert q == 1 and m >= 2 * L - 1 and D == 1
        else:
            assert -(-L // m) <= pc
            assert D == (q if dm == 0 else 1)
        if (m, D) in seen:
            continue
        seen.add((m, D))
        back = predict.class_index(L, M, m, D)
        assert predict.params_of(back, L, M, outer=False) == (m, D)


def test_outer_axes_respect_column_limit():
    for ci in range(len(predict.CLASSES)):
        m, _ = predict.params_of(ci, 8192, 16383, outer=True)
        assert m <= predict.MAX_OUTER_M


def test_features_encoding():
    f = predict.features([4096, 256], 1, "c128", batch=4)
    assert f.shape == (predict.D_IN,)
    assert f[0] == pytest.approx(8 / 16) and f[1] == pytest.approx(12 / 16) and f[2] == 0.0
    assert list(f[3:6]) == [0, 1, 0] and list(f[6:9]) == [0, 1, 0]
    assert f[9] == 1.0 and f[10] == pytest.approx(2 / 16)
    assert f[11] == pytest.approx(np.log2(4096 * 256 * 4) / 32)


def test_soft_target_weights():
    table = [((1024, 2), 1.00), ((512, 4), 1.03), ((256, 8), 1.5)]
    t = predict.soft_target(1000, 1999, table, outer=False)
    assert t.sum() == pytest.approx(1.0)
    i1 = predict.class_index(1000, 1999, 1024, 2)
    i2 = predict.class_index(1000, 1999, 512, 4)
    assert t[i1] > t[i2] > 0 and t[i1] / t[i2] == pytest.approx(np.e, rel=1e-3)


def test_training_problems_within_bound():
    """At most 2^20 elements, except the listed large 2D/3D problems (at most 2^26),
    none of which is an evaluation problem."""
    probs = predict.training_problems()
    assert len(probs) > 100
    large = {tuple(d) for d in predict.LARGE_PROBLEMS}
    for Ls, batch, dt in probs:
        n = int(np.prod(Ls)) * batch
        assert n <= (1 << 20) or (tuple(Ls) in large and batch == 1 and n <= (1 << 26))
        assert dt in ("c64", "c128") and 1 <= len(Ls) <= 3
    assert not large & {tuple(L) for L, _ in predict.EVAL_PROBLEMS}


def uneq_cost(Lf, Lg, M, m, lam, D, dtype):
    """A bowl with its minimum at Lambda m = 2^ceil(log2 Lg) / 2 and m = 64."""
    mg = m * lam
    return 1.0 + (math.log2(mg) - (math.log2(tune.pow2_ceil(Lg)) - 1)) ** 2 + 0.3 * (math.log2(m) - 6) ** 2


def test_uneq_candidates_admissible():
    cands = tune.uneq_candidates(12, 100000, 100011)
    assert cands
    for m, lam, D in cands:
        s, l, _ = hdc.uneq_derive(12, 100000, 100011, m, lam, 1, D)
        assert l["p"] <= 4 or l["q"] == 1
        assert s["p"] <= 16 and lam <= 1024 and l["m"] == m * lam


def test_uneq_a0_and_a1_find_the_model_argmin():
    t0 = tune.TunerUneq(tune.TuneDB(None), timer=uneq_cost)
    r0 = t0.a0(12, 100000, 100011)
    assert r0.params["m"] == 64 and r0.params["m"] * r0.params["lam"] == 65536
    calls = []

    def counting(*a):
        calls.append(a)
        return uneq_cost(*a)
    db = tune.TuneDB(None)
    t1 = tune.TunerUneq(db, timer=counting, seed=3)
    for Lg in (30000, 60000):
        t1.a1(12, Lg, Lg + 11)
    calls.clear()
    r1 = t1.a1(12, 100000, 100011)
    assert r1.params == r0.params
    assert len(calls) < len(tune.uneq_candidates(12, 100000, 100011))
    assert t1.a1(12, 100000, 100011).source == "db"


def test_uneq_nd_separable_finds_per_axis_argmin():
    """With a cost separable over axes, the per-axis search returns each axis's argmin."""
    sf, sg = (12, 12), (4096, 2000)
    M = [a + b - 1 for a, b in zip(sf, sg)]
    want = [(64, 16), (16, 64)]

    def cost(m, lam):
        t = 1.0
        for ax in range(2):
            if m[ax]:
                t += (math.log2(m[ax]) - math.log2(want[ax][0])) ** 2 + (math.log2(lam[ax]) - math.log2(want[ax][1])) ** 2
        return t
    for ax in range(2):
        assert want[ax] in tune.uneq_nd_candidates(sf, sg, M, ax)
    m, lam, n = tune.uneq_nd_separable(sf, sg, M, timer=cost)
    assert list(zip(m, lam)) == want and n > 4


def test_batch_tuner_picks_each_buckets_argmin():
    """Per-bucket A0 for an uneven batch: with a synthetic cost whose best FFT size is the
    next power of two up to L = 4096 and half of it beyond (p = 2), every group gets its
    argmin; ties go to the larger m."""
    Ls = [70, 100, 300, 1000, 3000, 5000, 7000, 9000, 20000, 40000, 64, 65536]
    calls = []

    def cost(ls, ms, dtype):
        calls.append((tuple(ls), ms[0]))
        tot = 0.0
        for L, m in zip(ls, ms):
            p = -(-L // m)
            want = 1 if L <= 4096 else 2
            tot += 1.0 + abs(p - want) + (0.0 if m >= 2 else 5.0)
        return tot
    choice, tables = tune.tune_batch(Ls, "c64", timer=cost)
    for L, m in zip(Ls, choice):
        p = -(-L // m)
        assert p == (1 if L <= 4096 else 2), (L, m)
        assert m == tune.pow2_ceil(L) >> (p - 1)
    # every group timed its 4 candidates (plus the library default when it is not
    # among them) once, on its own problems only
    groups = {tune.pow2_ceil(L) for L in Ls}
    want = {g: 4 + (tune.batch_default_m(g) not in [g >> j for j in range(4)]) for g in groups}
    assert set(tables) == groups and all(len(t) == want[g] for g, t in tables.items())
    assert len(calls) == sum(want.values())
    assert all(tune.batch_default_m(g) == (g if g != 8192 else 4096) for g in groups)
    # a flat cost: the larger m wins the tie
    choice, _ = tune.tune_batch([300, 5000], "c64", timer=lambda ls, ms, dt: 1.0)
    assert choice == [512, 8192]


def test_batch_tuning_database(tmp_path):
    """The per-bucket search recorded in a JSON-lines database (hdc_batch_db_record)
    gives back, through the library's host-only reader (hdc_batch_db_choose, the
    choice of hdc_batch_plan_db), exactly the FFT sizes the search returned; rows of
    another device or build, of the other dtype and of unrelated kinds are ignored;
    problems whose output is not 2L - 1, and buckets without a row, take the default;
    equal times go to the larger m; a line cut short by a kill is skipped."""
    db = str(tmp_path / "batch.jsonl")
    with open(db, "w") as fh:  # an unrelated row and a torn record
        fh.write(json.dumps({"key": json.dumps({"L": [64], "M": [127], "batch": 1, "dtype": "c64"}),
                             "params": {"D": 1, "m": 64}, "ms": 0.1, "device": "dev", "build": "b1"}) + "\n")
        fh.write('{"key": "{\\"bucket\\": 512')
    Ls = [70, 100, 300, 1000, 3000, 5000, 7000, 9000, 20000, 40000, 64, 65536]

    def cost(ls, ms, dtype):
        tot = 0.0
        for L, m in zip(ls, ms):
            p = -(-L // m)
            tot += 1.0 + abs(p - (1 if L <= 4096 else 2))
        return tot
    choice, tables = tune.tune_batch(Ls, "c64", timer=cost, db=db, device="dev", build="b1")
    assert tune.batch_db_choose(Ls, "c64", db, device="dev", build="b1") == choice
    rows = []
    for x in open(db):
        try:
            r = json.loads(x)
        except json.JSONDecodeError:
            continue  # the torn record
        if "bucket" in json.loads(r["key"]):
            rows.append(r)
    assert len(rows) == sum(len(t) for t in tables.values())
    # the other device/build/dtype sees only defaults
    dflt = [tune.batch_default_m(L) for L in Ls]
    assert tune.batch_db_choose(Ls, "c64", db, device="other", build="b1") == dflt
    assert tune.batch_db_choose(Ls, "c64", db, device="dev", build="b2") == dflt
    assert tune.batch_db_choose(Ls, "c128", db, device="dev", build="b1") == dflt
    assert tune.batch_db_choose(Ls, "c64", None) == dflt
    # first-outputs problems keep the default; a bucket without rows too
    Ms = [2 * L - 1 for L in Ls]
    Ms[8] = Ls[8]
    got = tune.batch_db_choose(Ls + [200000], "c64", db, Ms=Ms + [399999], device="dev", build="b1")
    assert got[:8] == choice[:8] and got[8] == dflt[8] and got[9:12] == choice[9:] \
        and got[12] == tune.batch_default_m(200000)
    # a later, faster row wins; an equal time goes to the larger m
    lib = hdc._lib.lib()
    assert lib.hdc_batch_db_record(db.encode(), 1024, 0, 256, 0.0, b"dev", b"b1") == 0
    assert tune.batch_db_choose([1000], "c64", db, device="dev", build="b1") == [256]
    assert lib.hdc_batch_db_record(db.encode(), 1024, 0, 512, 0.0, b"dev", b"b1") == 0
    assert tune.batch_db_choose([1000], "c64", db, device="dev", build="b1") == [512]
    # a recorded m that a problem cannot take (here not 7-smooth) leaves it at the default
    assert lib.hdc_batch_db_record(db.encode(), 2048, 0, 11, 0.0, b"dev", b"b1") == 0
    assert tune.batch_db_choose([1500], "c64", db, device="dev", build="b1") == [tune.batch_default_m(1500)]
    # bad records are refused
    assert lib.hdc_batch_db_record(db.encode(), 1000, 0, 256, 1.0, b"dev", b"b1") == 1  # not a power of two
    assert lib.hdc_batch_db_record(db.encode(), 1024, 0, 0, 1.0, b"dev", b"b1") == 1
    assert lib.hdc_batch_db_record(db.encode(), 1024, 0, 256, -1.0, b"dev", b"b1") == 1


def test_malformed_database_rows_are_skipped(tmp_path):
    """Rows a hand edit or a foreign writer could leave -- sizes beyond range (1e30 would
    overflow a 64-bit conversion), fractional sizes, missing fields, non-objects, nesting
    deep enough to exhaust a recursive parser's stack -- are skipped by the library's readers (bucket rows and tuner rows) and by TuneDB."""
    db = str(tmp_path / "bad.jsonl")
    bkey = json.dumps({"bucket": 1024, "dtype": "c64"})
    pkey = json.dumps({"L": [1000], "M": [1999], "batch": 1, "dtype": "c64"}, sort_keys=True)
    bad = [{"key": bkey, "params": {"m": 1e30}, "ms": 0.1}, {"key": bkey, "params": {"m": 256.5}, "ms": 0.1},
           {"key": json.dumps({"bucket": 1e30, "dtype": "c64"}), "params": {"m": 256}, "ms": 0.1},
           {"key": bkey, "params": {"m": 256}},
           {"key": pkey, "params": {"D": 1e30, "m": 1024}, "ms": 0.1},
           {"key": pkey, "params": {"D": 2, "m": [1e30]}, "ms": 0.1},
           {"key": pkey, "params": {"D": 2, "m": 1024, "tile": 1e12}, "ms": 0.1},
           {"params": {"D": 2, "m": 1024}, "ms": 0.1}, [1, 2], "text", 7]
    with open(db, "w") as fh:
        for r in bad:
            if isinstance(r, dict):
                r = dict(r, device="dev", build="b1")
            fh.write(json.dumps(r) + "\n")
        fh.write("[" * 100000 + "\n" + '{"a": ' * 100000 + "\n")  # nesting deeper than any row
    assert tune.batch_db_choose([1000], "c64", db, device="dev", build="b1") == [tune.batch_default_m(1000)]
    tdb = tune.TuneDB(db, device="dev", build="b1")
    assert all(isinstance(r, dict) and "key" in r for r in tdb.rows)
    res = tune.Tuner1D(tdb, timer=cost_model).a1(1000, 1999, "c64")
    assert res.source == "A1" and 128 <= res.params["m"] <= 512  # a search ran: no malformed row was taken


def test_checkpoint_format_and_training_range(tmp_path):
    """save_checkpoint writes the layout hdc_predictor_load reads: magic, format 2,
    layer sizes, float32 weights, then the per-feature training range."""
    import struct
    r = np.random.default_rng(0)
    params = [(r.normal(size=(5, predict.D_IN)), r.normal(size=5)), (r.normal(size=(16, 5)), r.normal(size=16))]
    lo, hi = np.zeros(predict.D_IN), np.ones(predict.D_IN)
    path = str(tmp_path / "net.bin")
    predict.save_checkpoint(path, params, lo, hi)
    raw = open(path, "rb").read()
    assert raw[:8] == b"HDCMLP01"
    ver, n = struct.unpack("<ii", raw[8:16])
    sizes = struct.unpack("<3i", raw[16:28])
    assert (ver, n, sizes) == (2, 2, (predict.D_IN, 5, 16))
    w = np.frombuffer(raw[28:], dtype="<f4")
    assert w.size == 5 * predict.D_IN + 5 + 16 * 5 + 16 + 2 * predict.D_IN
    assert np.allclose(w[:5 * predict.D_IN], params[0][0].ravel().astype(np.float32))
    assert np.array_equal(w[-2 * predict.D_IN:], np.concatenate([lo, hi]).astype(np.float32))
    x = np.full(predict.D_IN, 0.5)
    assert predict.in_range(x, lo, hi)
    x[3] = 1.0 + 2 * predict.RANGE_MARGIN
    assert not predict.in_range(x, lo, hi)
    assert predict.in_range(x, None, None)


def test_evaluation_problems_lie_inside_the_training_range():
    """The large training problems (up to 2^26 elements) bring the 2D/3D evaluation
    problems inside the range, so the network answers for them, without any of them
    being trained on; the held-out problems stay inside it too."""
    rows = []
    for Ls, batch, dt in predict.training_problems():
        rows += [predict.features(Ls, a, dt, batch) for a in range(len(Ls))]
    X = np.stack(rows)
    lo, hi = X.min(0), X.max(0)
    for Ls, dt in predict.EVAL_PROBLEMS:
        assert all(predict.in_range(predict.features(Ls, a, dt), lo, hi) for a in range(len(Ls))), Ls
    for Ls, dt in predict.HELDOUT_PROBLEMS:
        assert all(predict.in_range(predict.features(Ls, a, dt), lo, hi) for a in range(len(Ls))), Ls
