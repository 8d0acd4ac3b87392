"""Mixed-radix residue transforms: m = R 2^k with R odd and 7-smooth (section
3.1's FFT-friendly sizes) on the fused kernel, which splits each m-point DFT
into R sub-transforms of 2^k points and a direct R-point stage.  Against the
oracle's padded FFT in both dtypes: several input blocks with a ragged last
one, first outputs (M < 2L - 1), a zero tail, residues in several rounds per
workgroup (q beyond the residues that run side by side), copies,
autoconvolution, the largest odd factor (63) and sub-transform (1024), exact
Gaussian-integer results, batches with such m per bucket, and plan-to-plan
agreement with a power-of-two m."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import NP_DT, TOL, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")

FUSED_LDS = 81920  # per-row LDS budget of the fused kernel


def _fits(L, M, m, dtype):
    """The fused kernel's LDS rule (q residues of m + m/8 slots + q twiddles)."""
    q = -(-max(M, 2 * L - 1) // m)
    b = 16 if dtype == "c128" else 8
    return q * (m + m // 8) * b + q * 16 + 16 <= FUSED_LDS


def _ref(f64, g64, M):
    L = len(f64)
    full = oracle.padded_1d(f64, g64, max(M, 2 * L - 1))
    return full[:M]


def _run(L, M, m, dtype, C=1, cfg=950, idx=0, same=False):
    plan = hdc.Plan(L, M, m, C=C, dtype=dtype)
    ax = plan.axes[0]
    say(f"mixed L={L} M={M} m={m} p={ax['p']} q={ax['q']} C={C} {dtype} same={same} variant={ax['variant']}")
    assert ax["variant"] == 0 and ax["m"] == m
    f, g, f64, g64 = inputs(L if C == 1 else (L, C), cfg, idx, dtype)
    if same:
        g, g64 = f, f64
    ft = to_dev(f)
    h = to_host(plan.convolve(ft, ft if same else to_dev(g)))
    if C == 1:
        ref = _ref(f64, g64, M)
    else:
        ref = np.stack([_ref(f64[:, c], g64[:, c], M) for c in range(C)], axis=1)
    err = rel(h, ref)
    say(f"   rel={err:.3e}")
    assert err <= TOL[dtype], err
    if M > 2 * L - 1:  # the tail is zero up to the transform's rounding
        assert np.max(np.abs(h[2 * L - 1:])) <= TOL[dtype] * np.max(np.abs(ref))
    return h


MS = [3, 5, 6, 7, 12, 96, 320, 448, 9 * 8, 15 * 4, 21 * 16, 25 * 8, 27 * 2, 35 * 32, 45 * 16, 49 * 4, 63 * 16]
CASES = []
for m in MS:
    for L, M in ((m - 1 if m > 1 else 1, None), (2 * m + 1, None), (5 * m - 3, None), (5 * m - 3, 3 * m + 1),
                 (2 * m + 1, 6 * m + 5)):
        M = 2 * L - 1 if M is None else M
        for dt in ("c128", "c64"):
            if _fits(L, M, m, dt):
                CASES.append((L, M, m, dt))


@pytest.mark.parametrize("L,M,m,dtype", CASES)
def test_mixed_m_against_oracle(L, M, m, dtype):
    _run(L, M, m, dtype, idx=L + m)


@pytest.mark.parametrize("L,m,dtype", [(2237, 448, "c64"), (2555, 320, "c64"), (2100, 96, "c128"),
                                        (2000, 720, "c64")])
def test_residues_in_several_rounds(L, m, dtype):
    """q beyond the residues that run side by side (512 threads / (R 2^k / points
    per thread)): the workgroup takes its residues in several rounds."""
    R = m
    while R % 2 == 0:
        R //= 2
    p2 = m // R
    tpf = R * (p2 // min(p2, 8))
    q = -(-(2 * L - 1) // m)
    assert q > 512 // tpf and _fits(L, 2 * L - 1, m, dtype)
    _run(L, 2 * L - 1, m, dtype, idx=7)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,C,m", [(100, 3, 12), (700, 2, 96), (37, 4, 5)])
def test_copies(L, C, m, dtype):
    _run(L, 2 * L - 1, m, dtype, C=C, idx=C)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m", [(1000, 96), (2000, 448)])
def test_autoconvolution(L, m, dtype):
    _run(L, 2 * L - 1, m, dtype, same=True, idx=3)


@pytest.mark.parametrize("L,M,m,dtype", [(3000, 5999, 63 * 64, "c64"),    # R = 63, 504 threads per residue
                                         (2000, 3999, 3 * 1024, "c64"),   # the largest sub-transform
                                         (1500, 2999, 3 * 1024, "c128"),
                                         (1, 1, 3, "c128"), (2, 3, 7, "c64")])
def test_extremes(L, M, m, dtype):
    _run(L, M, m, dtype, idx=11)


@pytest.mark.parametrize("m", [3, 96, 320, 63 * 16])
def test_gaussian_integers_exact(m):
    L = 4 * m + 5 if _fits(4 * m + 5, 8 * m + 9, m, "c128") else m + 5
    f = synth.gaussian_integers(L, 8, 951, 0, 0)
    g = synth.gaussian_integers(L, 8, 951, 0, 1)
    exact = oracle.direct_1d(f, g, 2 * L - 1)
    plan = hdc.Plan(L, 2 * L - 1, m, dtype="c128")
    out = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert np.array_equal(np.round(out), exact)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_agrees_with_power_of_two_plan(dtype):
    """The same convolution from m = 96 and m = 128 (and deterministic replays)."""
    L = 2000
    f, g, _, _ = inputs(L, 952, 0, dtype)
    ft, gt = to_dev(f), to_dev(g)
    a = to_host(hdc.Plan(L, 2 * L - 1, 96, dtype=dtype).convolve(ft, gt))
    a2 = to_host(hdc.Plan(L, 2 * L - 1, 96, dtype=dtype).convolve(ft, gt))
    b = to_host(hdc.Plan(L, 2 * L - 1, 128, dtype=dtype).convolve(ft, gt))
    assert np.array_equal(a, a2)
    assert rel(a, b) <= 2 * TOL[dtype]


def test_stage_entry_points_reject_mixed_m():
    import torch
    plan = hdc.Plan(100, 199, 12, dtype="c64")
    x = torch.zeros(100, dtype=torch.complex64, device="cuda")
    with pytest.raises(hdc.HdcError):
        plan.forward(x, plan.residue_buffer(), 0)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_with_mixed_buckets(dtype):
    """A batch whose buckets take m = 3 2^k, 5 2^k, 7 2^k next to power-of-two
    buckets; every problem against the oracle, the graph replay equal to the
    eager launches."""
    import torch
    r = synth.rng(953, 0, 0)
    Ls = [int(x) for x in r.integers(1, 3000, 40)] + [1, 2, 5000]
    choices = (3, 12, 96, 320, 448, 0)
    bm = []
    for i, L in enumerate(Ls):
        m = choices[i % len(choices)]
        bm.append(m if m and _fits(L, 2 * L - 1, m, dtype) else 0)
    Ms = [2 * L - 1 for L in Ls]
    fs = [synth.uniform_complex(L, 953, i, 0, NP_DT[dtype]) for i, L in enumerate(Ls)]
    gs = [synth.uniform_complex(L, 953, i, 1, NP_DT[dtype]) for i, L in enumerate(Ls)]
    fp, gp = to_dev(np.concatenate(fs)), to_dev(np.concatenate(gs))
    B = hdc.Batch(Ls, bucket_m=bm, dtype=dtype)
    say(f"batch mixed n={len(Ls)} buckets={B.n_buckets} {dtype}")
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
