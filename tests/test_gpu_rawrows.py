"""The raw-residue-row path (variant 2): residue transforms of one row (m <= 4096)
formed from the raw inputs (eq. (3)'s block sums) inside the row kernel, with
the output sums of eq. (4) over q <= 32 residues in a second kernel.  Against
the oracle's padded FFT in both dtypes: p from 2 to 4, q up to the limit of
32, residue groups (D < q, the output accumulated), copies, first outputs
(M < 2L - 1), a zero tail (M > 2L - 1), autoconvolution; q = 33 or p = 5 fall
back to the column/row/column passes.  Batches: several m served by raw groups
next to fused and column/row buckets."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import NP_DT, TOL, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")
from paper_2306_10016_amd import tune  # noqa: E402

# (L, M, m, D, C)
CASES = [
    (5000, 9999, 4096, 0, 1),       # p = 2, q = 3
    (16384, 131072, 4096, 0, 1),    # p = 4, q = 32: the limit (outputs beyond 2L - 1 are zero)
    (16384, 131072, 4096, 8, 1),    # four groups of 8, the output accumulated
    (8000, 15999, 2048, 1, 2),      # p = 4, q = 8, one residue per group, two copies
    (6000, 6000, 2048, 0, 1),       # first outputs: q = 6 from 2L - 1, 3 output blocks
    (6000, 20000, 2048, 0, 1),      # q = 10, a zero tail
    (12000, 23999, 4096, 0, 3),     # p = 3, q = 6, three copies
    (7000, 13999, 2048, 5, 1),      # q = 7 in groups of 5 (the last one short)
]


def _ref(f64, g64, M, C):
    if C == 1:
        return oracle.padded_1d(f64, g64, M) if M >= 2 * len(f64) - 1 else oracle.padded_1d(f64, g64, 2 * len(f64) - 1)[:M]
    return np.stack([_ref(f64[:, c], g64[:, c], M, 1) for c in range(C)], axis=1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,M,m,D,C", CASES)
def test_raw_rows_against_oracle(L, M, m, D, C, dtype):
    plan = hdc.Plan(L, M, m, D=D, C=C, dtype=dtype)
    ax = plan.axes[0]
    say(f"raw rows L={L} M={M} m={m} p={ax['p']} q={ax['q']} D={ax['D']} C={C} {dtype} variant={ax['variant']}")
    assert ax["variant"] == 2 and ax["m1"] == 1
    f, g, f64, g64 = inputs(L if C == 1 else (L, C), 900, L % 101 + C, dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    ref = _ref(f64, g64, M, C)
    err = rel(h, ref)
    say(f"   rel={err:.3e}")
    assert err <= TOL[dtype], err
    if M > 2 * L - 1:  # the tail is zero up to the transform's rounding
        assert np.max(np.abs(h[2 * L - 1:])) <= TOL[dtype] * np.max(np.abs(ref))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_raw_rows_autoconvolution_and_determinism(dtype):
    L, m = 7000, 2048
    f, _, f64, _ = inputs(L, 901, 0, dtype)
    plan = hdc.Plan(L, 2 * L - 1, m, dtype=dtype)
    assert plan.axes[0]["variant"] == 2
    ft = to_dev(f)
    a = to_host(plan.convolve(ft, ft))
    b = to_host(plan.convolve(ft, ft))
    assert np.array_equal(a, b)
    assert rel(a, oracle.padded_1d(f64, f64, 2 * L - 1)) <= TOL[dtype]


def test_raw_rows_gaussian_integers_exact():
    L = 4096 * 3 + 17
    f = synth.gaussian_integers(L, 8, 902, 0, 0)
    g = synth.gaussian_integers(L, 8, 902, 0, 1)
    exact = oracle.direct_1d(f, g, 2 * L - 1)
    plan = hdc.Plan(L, 2 * L - 1, 4096, dtype="c128")
    assert plan.axes[0]["variant"] == 2
    out = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert np.array_equal(np.round(out), exact)


@pytest.mark.parametrize("L,M", [(4 * 4096, 33 * 4096), (4 * 4096 + 1, 8 * 4096 + 1)])
def test_beyond_the_limits_takes_the_column_path(L, M):
    plan = hdc.Plan(L, M, 4096, dtype="c64")
    ax = plan.axes[0]
    assert (ax["q"] == 33 or ax["p"] == 5) and ax["variant"] == 1
    f, g, f64, g64 = inputs(L, 903, 0, "c64")
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert rel(h, _ref(f64, g64, M, 1)) <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_raw_groups_of_several_m(dtype):
    """A batch whose raw groups have m = 512, 2048 and 4096 (p up to 4), beside
    fused and column/row/column buckets; every problem against the oracle, and the
    graph replay equal to the eager launches."""
    import torch
    r = synth.rng(904, 0, 0)
    Ls = [int(x) for x in r.integers(600, 65536, 60)] + [70, 300, 1000, 100000, 140000]
    bm = []
    for L in Ls:
        fits = [m for m in (512, 2048, 4096) if -(-L // m) <= 4]
        if L <= 1000:
            bm.append(0)            # the fused kernel
        elif fits:
            bm.append(fits[L % len(fits)])  # raw groups (or the fused kernel where it fits)
        else:
            bm.append(0)            # column/row/column
    Ms = [2 * L - 1 for L in Ls]
    fs = [synth.uniform_complex(L, 904, i, 0, NP_DT[dtype]) for i, L in enumerate(Ls)]
    gs = [synth.uniform_complex(L, 904, i, 1, NP_DT[dtype]) for i, L in enumerate(Ls)]
    fp, gp = to_dev(np.concatenate(fs)), to_dev(np.concatenate(gs))
    B = hdc.Batch(Ls, bucket_m=bm, dtype=dtype)
    say(f"batch raw groups n={len(Ls)} buckets={B.n_buckets} {dtype}")
    eager = torch.empty(B.total_M, dtype=fp.dtype, device="cuda")
    B.convolve(fp, gp, eager, graph=False)
    out = torch.empty_like(eager)
    for rep in range(2):
        out.fill_(float("nan"))
        B.convolve(fp, gp, out, graph=True)
        torch.cuda.synchronize()
        rv = torch.float64 if dtype == "c128" else torch.float32
        assert torch.equal(out.view(rv), eager.view(rv)), rep
    h = to_host(eager)
    offs = np.concatenate([[0], np.cumsum(Ms)])
    for i in range(len(Ls)):
        ref = oracle.padded_1d(fs[i].astype(np.complex128), gs[i].astype(np.complex128), Ms[i])
        assert rel(h[offs[i]:offs[i + 1]], ref) <= TOL[dtype], (i, Ls[i], bm[i])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_queue_equals_single_plans(dtype):
    """Problems the persistent fused launch serves (every fused size, several blocks
    of problems per bucket) and raw-group problems give the same bits as single
    plans of the same parameters."""
    import torch
    Ls = [1, 3, 17, 64, 100, 500, 1000, 1500, 3000, 4096, 5000, 20000, 65536]
    Ls = [L for L in Ls for _ in range(3)]
    Ms = [2 * L - 1 for L in Ls]
    fs = [synth.uniform_complex(L, 905, i, 0, NP_DT[dtype]) for i, L in enumerate(Ls)]
    gs = [synth.uniform_complex(L, 905, i, 1, NP_DT[dtype]) for i, L in enumerate(Ls)]
    B = hdc.Batch(Ls, dtype=dtype)
    say(f"batch queue vs single plans {dtype} buckets={B.n_buckets}")
    out = to_host(B.convolve(to_dev(np.concatenate(fs)), to_dev(np.concatenate(gs))))
    offs = np.concatenate([[0], np.cumsum(Ms)])
    for i, L in enumerate(Ls):
        m = tune.batch_default_m(L)
        single = to_host(hdc.Plan(L, Ms[i], m, dtype=dtype).convolve(to_dev(fs[i]), to_dev(gs[i])))
        assert np.array_equal(out[offs[i]:offs[i + 1]], single), (i, L, m)
