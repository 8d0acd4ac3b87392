"""GPU parity of unequal extents in 2D/3D (section 3.6 with section 3.5's
lengths) against the FP64 oracle, element by element on small boxes and on
sampled outputs at full size."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, NP_DT, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CFG = 650

CASES = [
    # (f extents, g extents, m per axis or None, Lambda per axis or None, D per axis or None)
    ((12, 12), (100, 90), None, None, None),
    ((12, 12), (100, 90), (16, 16), (4, 8), (2, 0)),
    ((3, 50), (40, 4), None, None, None),                 # f shorter on x, longer on y
    ((60, 2), (5, 70), (8, 4), (16, 32), (3, 1)),
    ((7, 9), (300, 250), (32, 16), (16, 32), (0, 3)),
    ((12, 12), (200, 200), (64, 256), (4, 1), None),      # Lambda = 1 on the inner axis: fused rows
    ((12, 30), (200, 9000), (64, 4096), (4, 1), None),    # Lambda = 1 inner, too large to fuse: raw rows
    ((6, 10), (30, 300), (8, 16), (2, 4), (2, 2)),        # several residues and groups on both axes
    ((5, 8), (3000, 20), (8, 8), (512, 4), None),         # outer Lambda m = 4096: two column stages
    ((100, 6), (2500, 40), (128, 8), (16, 8), (2, 0)),    # outer m1f = 64 > 1 and p_g > 1
    ((3, 5, 7), (20, 21, 22), None, None, None),
    ((2, 2, 2), (30, 40, 50), (4, 4, 4), (8, 16, 16), (1, 2, 0)),
    ((9, 3, 12), (4, 30, 5), None, None, None),           # roles differ per axis
]


def _ops(sf, sg, dtype, idx):
    f = synth.uniform_complex(sf, CFG, idx, 0, NP_DT[dtype])
    g = synth.uniform_complex(sg, CFG, idx, 1, NP_DT[dtype])
    return f, g


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", CASES, ids=[f"{'x'.join(map(str, c[0]))}_{'x'.join(map(str, c[1]))}_{i}"
                                             for i, c in enumerate(CASES)])
def test_uneq_nd_matches_oracle(case, dtype):
    import paper_2306_10016_amd as hdc
    sf, sg, m, lam, D = case
    idx = CASES.index(case)
    M = [a + b - 1 for a, b in zip(sf, sg)]
    say(f"uneq nd f={sf} g={sg} m={m} lam={lam} D={D} {dtype}")
    plan = hdc.UneqPlan.nd(sf, sg, M, m=m, lam=lam, D=D, dtype=dtype)
    f, g = _ops(sf, sg, dtype, idx)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    ref = oracle.padded_nd(f.astype(np.complex128), g.astype(np.complex128), M)
    err = rel(h, ref)
    say(f"  long={[(a['m'], a['m1'], a['m2'], a['q'], a['variant']) for a in plan.axes]} "
        f"short={[(a['m'], a['m1'], a['m2'], a['q']) for a in plan.short_axes]} err={err:.2e}")
    assert h.shape == tuple(M)
    assert err < TOL[dtype]


def test_uneq_nd_longer_output_box():
    """M beyond Lf + Lg - 1 on every axis: the tail is zero."""
    import paper_2306_10016_amd as hdc
    sf, sg = (4, 6), (50, 33)
    M = (60, 45)
    plan = hdc.UneqPlan.nd(sf, sg, M, m=(8, 8), lam=(8, 4), dtype="c128")
    f, g = _ops(sf, sg, "c128", 40)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert rel(h, oracle.padded_nd(f, g, M)) < TOL["c128"]
    assert np.all(np.abs(h[53:, :]) < 1e-13) and np.all(np.abs(h[:, 38:]) < 1e-13)


def test_uneq_nd_integer_exact():
    import paper_2306_10016_amd as hdc
    sf, sg = (5, 7), (60, 80)
    f = synth.gaussian_integers(sf, 8, CFG, 41, 0)
    g = synth.gaussian_integers(sg, 8, CFG, 41, 1)
    plan = hdc.UneqPlan.nd(sf, sg, dtype="c128")
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    ref = oracle.direct_nd(f, g, [64, 86])
    assert np.array_equal(np.round(h), ref)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_uneq_nd_full_size_sampled(dtype):
    """A 12 x 12 filter against a 4096 x 4096 image, checked at sampled outputs
    (corners, edges, block boundaries, random interior points)."""
    import paper_2306_10016_amd as hdc
    sf, sg = (12, 12), (4096, 4096)
    M = [a + b - 1 for a, b in zip(sf, sg)]
    plan = hdc.UneqPlan.nd(sf, sg, M, dtype=dtype)
    f, g = _ops(sf, sg, dtype, 50)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    r = synth.rng(CFG, 51, 0)
    pts = [(0, 0), (0, M[1] - 1), (M[0] - 1, 0), (M[0] - 1, M[1] - 1), (11, 11), (4095, 4095), (2048, 5)]
    pts += [tuple(int(v) for v in r.integers(0, M, 2)) for _ in range(300)]
    ks = np.array([i * M[1] + j for i, j in pts], dtype=np.int64)
    ref = oracle.direct_nd_sampled(f.astype(np.complex128), g.astype(np.complex128), M, ks)
    got = h.reshape(-1)[ks]
    err = rel(got, ref)
    say(f"  4096^2 x 12^2 {dtype}: long={plan.axes} err={err:.2e}")
    assert err < TOL[dtype]


def test_uneq_nd_deterministic():
    import paper_2306_10016_amd as hdc
    sf, sg = (9, 3, 12), (4, 30, 5)
    plan = hdc.UneqPlan.nd(sf, sg, dtype="c64")
    f, g = _ops(sf, sg, "c64", 60)
    fd, gd = to_dev(f), to_dev(g)
    assert np.array_equal(to_host(plan.convolve(fd, gd)), to_host(plan.convolve(fd, gd)))
