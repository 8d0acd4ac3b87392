"""GPU parity of the N-D passes (section 3.6) and of uneven-length batches."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, NP_DT, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")


def _nd(L, M, m, dtype, D=None, cfg=300, idx=0, full=True, nsample=48):
    say(f"nd L={L} M={M} m={m} D={D} {dtype}")
    f, g, f64, g64 = inputs(tuple(L), cfg, idx, dtype)
    plan = hdc.Plan.nd(L, M, m, D=D, dtype=dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert h.shape == tuple(M)
    if full:
        ref = oracle.padded_nd(f64, g64, M)
        err = rel(h, ref)
    else:
        r = synth.rng(cfg, idx, 5)
        tot = int(np.prod(M))
        ks = np.unique(np.concatenate([[0, tot - 1], r.integers(0, tot, nsample)]))
        ref = oracle.direct_nd_sampled(f64, g64, M, ks)
        err = rel(h.reshape(-1)[ks], ref)
    say(f"   rel={err:.3e}")
    assert err <= TOL[dtype], err
    return plan, h


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,extra,m,D", [((6, 9), (0, 0), (4, 8), None), ((16, 24), (0, 3), (8, 16), None),
                                         ((16, 24), (0, 0), (8, 16), (1, 2)), ((37, 50), (5, 0), (16, 32), (3, 0)),
                                         ((1, 50), (0, 0), (1, 64), None), ((50, 1), (0, 0), (64, 1), None),
                                         ((33, 700), (0, 0), (64, 1024), (1, 1)),
                                         # outer axes with several input blocks (p = 3), one split 1024 x 2
                                         ((3000, 50), (0, 0), (1024, 64), None), ((5000, 20), (0, 0), (2048, 32), None)])
def test_2d(L, extra, m, D, dtype):
    M = tuple(2 * a - 1 + e for a, e in zip(L, extra))
    _nd(L, M, m, dtype, D=D, idx=L[0])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m,D", [((8, 12, 10), (4, 8, 8), None), ((5, 6, 7), (2, 4, 8), (1, 2, 0)),
                                   ((9, 4, 33), (16, 2, 64), None), ((2500, 7, 30), (1024, 8, 32), None)])
def test_3d(L, m, D, dtype):
    M = tuple(2 * a - 1 for a in L)
    _nd(L, M, m, dtype, D=D, idx=L[2])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m", [((256, 256), (256, 256)), ((512, 512), (512, 512)), ((1024, 1024), (1024, 1024)),
                                 ((2048, 512), (1024, 512)), ((1024, 4096), (1024, 4096))])
def test_2d_workload_sizes_sampled(L, m, dtype):
    M = tuple(2 * a - 1 for a in L)
    _nd(L, M, m, dtype, idx=L[0] + L[1], full=False)


def test_3d_256_sampled():
    L = (256, 256, 256)
    _nd(L, tuple(2 * a - 1 for a in L), (256, 256, 256), "c64", idx=256, full=False, nsample=24)


def test_2d_separable():
    """f = a (x) b, g = c (x) d  =>  h = (a*c) (x) (b*d)."""
    a, c = synth.uniform_complex(40, 301, 0, 0), synth.uniform_complex(40, 301, 1, 0)
    b, d = synth.uniform_complex(70, 301, 2, 0), synth.uniform_complex(70, 301, 3, 0)
    f, g = np.outer(a, b), np.outer(c, d)
    plan = hdc.Plan.nd((40, 70), (79, 139), (32, 64), dtype="c128")
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    want = np.outer(oracle.padded_1d(a, c, 79), oracle.padded_1d(b, d, 139))
    assert rel(h, want) <= 1e-12


def test_2d_autoconvolution():
    f, _, f64, _ = inputs((60, 45), 302, 0, "c128")
    plan = hdc.Plan.nd((60, 45), (119, 89), (64, 32), dtype="c128")
    ft = to_dev(f)
    h = to_host(plan.convolve(ft, ft))
    assert rel(h, oracle.padded_nd(f64, f64, (119, 89))) <= 1e-12


def _batch(Ls, dtype, bucket_m=None, graph=True, cfg=310, check_idx=None, replays=1, tune_db=None):
    Ls = [int(x) for x in Ls]
    Ms = [2 * x - 1 for x in Ls]
    fs = [synth.uniform_complex(L, cfg, i, 0, NP_DT[dtype]) for i, L in enumerate(Ls)]
    gs = [synth.uniform_complex(L, cfg, i, 1, NP_DT[dtype]) for i, L in enumerate(Ls)]
    fp, gp = to_dev(np.concatenate(fs)), to_dev(np.concatenate(gs))
    B = hdc.Batch(Ls, bucket_m=bucket_m, dtype=dtype, tune_db=tune_db)
    say(f"batch n={len(Ls)} buckets={B.n_buckets} {dtype} graph={graph}")
    import torch
    out = torch.empty(B.total_M, dtype=fp.dtype, device="cuda")
    offs = np.concatenate([[0], np.cumsum(Ms)])
    idx = range(len(Ls)) if check_idx is None else check_idx
    refs = {i: oracle.padded_1d(fs[i].astype(np.complex128), gs[i].astype(np.complex128), Ms[i]) for i in idx}
    for rep in range(replays):
        out.fill_(float("nan"))
        B.convolve(fp, gp, out, graph=graph)
        h = to_host(out)
        tmp = torch.ones(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert float(tmp) == 1000.0
        for i in idx:
            err = rel(h[offs[i]:offs[i + 1]], refs[i])
            assert err <= TOL[dtype], (rep, i, Ls[i], err)
    return B


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_small_eager_and_graph(dtype):
    Ls = synth.batch_lengths(64, 3, 13, cfg=311)
    _batch(Ls, dtype, graph=False)
    _batch(Ls, dtype, graph=True, replays=3)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_bucket_override(dtype):
    Ls = synth.batch_lengths(40, 4, 12, cfg=312)
    bm = [max(1, int(2 ** np.floor(np.log2(L))) // 2) for L in Ls]  # p = 2 or 3 classes
    _batch(Ls, dtype, bucket_m=bm, graph=True, replays=2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_planned_from_tuning_database(dtype, tmp_path):
    """The per-bucket search timed on the GPU into a JSON-lines database; a batch planned
    from it (hdc_batch_plan_db) takes exactly the search's FFT sizes: the same buckets and
    bitwise the same output as the batch planned with those sizes, within the oracle's bar."""
    import torch
    from paper_2306_10016_amd import tune
    Ls = [int(x) for x in synth.batch_lengths(48, 5, 13, cfg=314)]
    db = str(tmp_path / "batch_db.jsonl")
    choice, tables = tune.tune_batch(Ls, dtype, db=db, reps=1)
    say(f"tuned {len(tables)} buckets: {[(s, min(t, key=lambda r: r[1])[0]) for s, t in sorted(tables.items())]}")
    assert tune.batch_db_choose(Ls, dtype, db) == choice
    Bd = _batch(Ls, dtype, tune_db=db, cfg=314, replays=2)
    Bc = hdc.Batch(Ls, bucket_m=choice, dtype=dtype)
    assert Bd.n_buckets == Bc.n_buckets
    fp = torch.randn(Bd.total_L, dtype=torch.complex128 if dtype == "c128" else torch.complex64, device="cuda")
    gp = torch.randn_like(fp)
    hd, hc = Bd.convolve(fp, gp), Bc.convolve(fp, gp)
    torch.cuda.synchronize()
    assert torch.equal(hd, hc)


def test_batch_edge_lengths():
    _batch([1, 2, 3, 1, 64, 65, 4096, 4097, 9000], "c128", graph=True, replays=2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_lanes_bitwise_equal_eager(dtype):
    """The graph runs the buckets on concurrent lanes, each with its own workspace
    region; every replay equals the eager launches (buckets in turn on one stream)
    bit for bit, and both match the oracle on sampled problems."""
    import torch
    Ls = [int(x) for x in synth.batch_lengths(240, 6, 15, cfg=313)]
    Ms = [2 * x - 1 for x in Ls]
    fp = to_dev(np.concatenate([synth.uniform_complex(L, 313, i, 0, NP_DT[dtype]) for i, L in enumerate(Ls)]))
    gp = to_dev(np.concatenate([synth.uniform_complex(L, 313, i, 1, NP_DT[dtype]) for i, L in enumerate(Ls)]))
    B = hdc.Batch(Ls, dtype=dtype)
    say(f"batch lanes n={len(Ls)} buckets={B.n_buckets} {dtype}")
    assert B.n_buckets >= 8
    eager = torch.empty(B.total_M, dtype=fp.dtype, device="cuda")
    B.convolve(fp, gp, eager, graph=False)
    out = torch.empty_like(eager)
    for rep in range(3):
        out.fill_(float("nan"))
        B.convolve(fp, gp, out, graph=True)
        tmp = torch.ones(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert float(tmp) == 1000.0
        assert torch.equal(out.view(torch.float64 if dtype == "c128" else torch.float32),
                           eager.view(torch.float64 if dtype == "c128" else torch.float32)), rep
    h = to_host(eager)
    offs = np.concatenate([[0], np.cumsum(Ms)])
    for i in sorted({int(np.argmax(Ls)), int(np.argmin(Ls)), 7, 100, 200}):
        ref = oracle.padded_1d(synth.uniform_complex(Ls[i], 313, i, 0, NP_DT[dtype]).astype(np.complex128),
                               synth.uniform_complex(Ls[i], 313, i, 1, NP_DT[dtype]).astype(np.complex128), Ms[i])
        assert rel(h[offs[i]:offs[i + 1]], ref) <= TOL[dtype], (i, Ls[i])


def test_batch_full_workload_sampled():
    """4096 complex64 problems, L log-uniform in [64, 65536]; 40 problems checked in full."""
    Ls = synth.batch_lengths(4096, 6, 16, cfg=3)
    check = sorted(set(synth.rng(3, 0, 6).integers(0, 4096, 36).tolist()) | {int(np.argmax(Ls)), int(np.argmin(Ls))})
    _batch(Ls, "c64", graph=True, cfg=3, check_idx=check, replays=2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m,D", [((3000, 40), (4096, 64), None), ((1500, 100), (2048, 128), (1, 0)),
                                   ((1100, 6, 5), (2048, 8, 8), None), ((700, 33), (8192, 64), (3, 0)),
                                   ((3000, 20), (2048, 32), None), ((3000, 20), (2048, 32), (2, 0))])
def test_outer_axis_four_step(L, m, D, dtype):
    """Outer axes with m > 1024 run as two column stages (m1 = 1024, then a strided m2-point pass);
    with q = 3 the backward columns take one group of three residues or groups of two and one
    (the second accumulating into h)."""
    M = tuple(2 * a - 1 for a in L)
    plan, _ = _nd(L, M, m, dtype, D=D, idx=L[0] + 7)
    assert plan.axes[0]["m1"] * plan.axes[0]["m2"] == m[0]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_inner_axis_many_rows(dtype):
    """Innermost axis with many rows: in complex64 one workgroup per row with the
    output sums in registers (m = 1024 .. 4096, q_out <= 4); otherwise one-row
    residues of 2048 points and more run a workgroup per (row, residue) on the
    raw-row path, and below that, with N beyond 80 KiB of LDS, the fused kernel
    takes the whole LDS of a workgroup."""
    plan, _ = _nd((64, 3000), (127, 5999), (64, 4096), dtype, idx=11)
    assert plan.axes[1]["variant"] == (3 if dtype == "c64" else 2)
    plan, _ = _nd((40, 9000), (79, 17999), (64, 4096), dtype, idx=13)
    assert plan.axes[1]["variant"] == 2 and plan.axes[1]["q_out"] == 5
    plan, _ = _nd((64, 1500), (127, 2999), (64, 1024), dtype, idx=12)
    assert plan.axes[1]["variant"] == (3 if dtype == "c64" else 0)


def test_column_batches_beyond_grid_limit():
    """(16, 4096, 16): the middle axis's strided pass runs 65536 column batches (> 65535 per launch)."""
    L = (16, 4096, 16)
    _nd(L, tuple(2 * a - 1 for a in L), (16, 4096, 16), "c64", idx=99, full=False, nsample=40)


def test_batch_inside_a_caller_capture():
    """hdc_batch_convolve refuses a capturing stream (it replays a graph of its own);
    hdc_batch_convolve_eager can be captured: every replay of the caller's graph, with
    eager work between replays, equals the eager result bit for bit."""
    import torch
    Ls = [int(x) for x in synth.batch_lengths(48, 6, 13, cfg=314)]
    fp = to_dev(np.concatenate([synth.uniform_complex(L, 314, i, 0, np.complex64) for i, L in enumerate(Ls)]))
    gp = to_dev(np.concatenate([synth.uniform_complex(L, 314, i, 1, np.complex64) for i, L in enumerate(Ls)]))
    B = hdc.Batch(Ls, dtype="c64")
    say(f"batch in capture n={len(Ls)} buckets={B.n_buckets}")
    ws = B.workspace()
    eager = B.convolve(fp, gp, ws=ws, graph=False).clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=s, capture_error_mode="thread_local"):
        with pytest.raises(hdc.HdcError) as e:
            B.convolve(fp, gp, out, ws=ws, stream=s, graph=True)
        B.convolve(fp, gp, out, ws=ws, stream=s, graph=False)
    assert e.value.status == 1 and "captured" in str(e.value)
    for rep in range(3):
        out.fill_(float("nan"))
        gr.replay()
        tmp = torch.ones(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert float(tmp) == 1000.0
        assert torch.equal(out.view(torch.float32), eager.view(torch.float32)), rep
