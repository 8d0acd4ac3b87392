"""GPU parity of the first-outputs mode: an output count M below the length of
the linear convolution (M = L is the backward range t < p of section 2.2).  The
transform still covers all 2L - 1 (or Lf + Lg - 1) terms; only the first M
outputs are written.  Reference: the oracle's direct sum over k < M.

The bar: relative L2 over the prefix itself, ||h - ref|| / ||ref|| over the M
outputs written, at the usual 1e-12 / 2e-6.  It is loosened only for short
prefixes, by the factor kappa = sqrt(M/K) ||full|| / ||prefix|| (K outputs in
the full linear convolution): the transform's rounding error is spread evenly
over its outputs, so a prefix of M of them carries about sqrt(M/K) of the
whole error, while its own norm is ||prefix|| / ||full|| of the whole; kappa
is the ratio of those shares (about 1 for M = L, about 20 for M = 1 of
L = 1000).  The bar is TOL max(1, kappa).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, NP_DT, inputs, say, to_dev, to_host


def rel(h, ref, full):
    """||h - ref|| / ||ref|| over the prefix, divided by max(1, kappa) (module docstring),
    so that it is compared with the plain bar TOL."""
    h, ref, full = np.ravel(h), np.ravel(ref), np.ravel(full)
    nref = np.linalg.norm(ref)
    kappa = np.sqrt(ref.size / full.size) * np.linalg.norm(full) / nref
    return float(np.linalg.norm(h - ref) / nref / max(1.0, kappa))

pytestmark = pytest.mark.gpu

CASES = [  # (L, M, m, D, C)
    (1000, 1000, 256, 0, 1), (1000, 1000, 256, 1, 1), (1000, 1, 64, 0, 1), (1000, 1998, 128, 3, 1),
    (37, 20, 8, 0, 1), (6, 6, 4, 1, 1), (3000, 3000, 8192, 0, 1), (5000, 2500, 1024, 2, 1),
    (6000, 6000, 8192, 1, 1), (300, 300, 64, 0, 3), (3000, 1500, 8192, 0, 2),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", CASES, ids=[f"L{c[0]}_M{c[1]}_m{c[2]}_D{c[3]}_C{c[4]}" for c in CASES])
def test_first_outputs_1d(case, dtype):
    import paper_2306_10016_amd as hdc
    L, M, m, D, C = case
    shape = L if C == 1 else (L, C)
    f, g, f64, g64 = inputs(shape, 800, CASES.index(case), dtype)
    plan = hdc.Plan(L, M, m, 0, 0, C, D, dtype)
    assert plan.axes[0]["N"] >= 2 * L - 1
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    ref = oracle.direct_1d(f64, g64, M)
    err = rel(h.reshape(ref.shape), ref, oracle.direct_1d(f64, g64, 2 * L - 1))
    say(f"first-M L={L} M={M} m={m} D={D} C={C} {dtype} variant={plan.axes[0]['variant']} err={err:.2e}")
    assert h.shape[0] == M and err < TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_first_outputs_full_size(dtype):
    """L = 2^22, M = L: the first half of the convolution, sampled."""
    import paper_2306_10016_amd as hdc
    L = 1 << 22
    f, g, f64, g64 = inputs(L, 801, 0, dtype)
    plan = hdc.Plan(L, L, L, dtype=dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    r = synth.rng(801, 1, 0)
    ks = np.unique(np.concatenate([np.arange(8), L - 8 + np.arange(8), r.integers(0, L, 200)]))
    ref = oracle.direct_1d_sampled(f64, g64, ks)
    assert h.shape == (L,) and rel(h[ks], ref, ref) < TOL[dtype]


def test_first_outputs_batch():
    import torch
    import paper_2306_10016_amd as hdc
    Ls = [int(x) for x in synth.batch_lengths(50, 3, 13, cfg=802)]
    Ms = [max(1, L // (1 + i % 3)) for i, L in enumerate(Ls)]
    fs = [synth.uniform_complex(L, 802, i, 0) for i, L in enumerate(Ls)]
    gs = [synth.uniform_complex(L, 802, i, 1) for i, L in enumerate(Ls)]
    B = hdc.Batch(Ls, M=Ms, dtype="c128")
    out = torch.empty(B.total_M, dtype=torch.complex128, device="cuda")
    offs = np.concatenate([[0], np.cumsum(Ms)])
    for graph in (False, True, True):
        out.fill_(float("nan"))
        B.convolve(to_dev(np.concatenate(fs)), to_dev(np.concatenate(gs)), out, graph=graph)
        h = to_host(out)
        for i in range(len(Ls)):
            full = oracle.direct_1d(fs[i], gs[i], 2 * Ls[i] - 1)
            assert rel(h[offs[i]:offs[i + 1]], full[:Ms[i]], full) < TOL["c128"], (i, Ls[i], Ms[i])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,M,m", [((64, 80), (64, 80), (64, 64)), ((100, 90), (100, 179), (32, 128)),
                                   ((40, 30, 20), (40, 30, 20), (16, 16, 16)), ((2048, 64), (2048, 64), (2048, 64))])
def test_first_outputs_nd(L, M, m, dtype):
    import paper_2306_10016_amd as hdc
    f, g, f64, g64 = inputs(L, 803, sum(L), dtype)
    plan = hdc.Plan.nd(list(L), list(M), list(m), dtype=dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    full = oracle.padded_nd(f64, g64, [2 * x - 1 for x in L])
    ref = full[tuple(slice(0, x) for x in M)]
    assert h.shape == tuple(M) and rel(h, ref, full) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_first_outputs_unequal(dtype):
    import paper_2306_10016_amd as hdc
    for i, (Lf, Lg, M, m, lam) in enumerate([(12, 1000, 1000, 16, 4), (12, 1000, 5, 16, 64), (300, 5000, 2000, 64, 32),
                                             (100, 2187, 2187, 128, 1)]):
        f = synth.uniform_complex(Lf, 804, i, 0, NP_DT[dtype])
        g = synth.uniform_complex(Lg, 804, i, 1, NP_DT[dtype])
        plan = hdc.UneqPlan(Lf, Lg, M, m=m, lam=lam, dtype=dtype)
        h = to_host(plan.convolve(to_dev(f), to_dev(g)))
        full = oracle.direct_1d(f.astype(np.complex128), g.astype(np.complex128), Lf + Lg - 1)
        assert h.shape == (M,) and rel(h, full[:M], full) < TOL[dtype], (Lf, Lg, M)
    sf, sg, M = (12, 12), (300, 200), (300, 200)
    f = synth.uniform_complex(sf, 805, 0, 0, NP_DT[dtype])
    g = synth.uniform_complex(sg, 805, 0, 1, NP_DT[dtype])
    plan = hdc.UneqPlan.nd(sf, sg, M, dtype=dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    full = oracle.padded_nd(f.astype(np.complex128), g.astype(np.complex128), (311, 211))
    assert h.shape == M and rel(h, full[:300, :200], full) < TOL[dtype]
