"""GPU parity of the real-data convolution (the real case that section 7 leaves
to future work): real f and g transformed together as z = f + i g, residue r
paired with q - r, only the residues r <= q/2 multiplied and inverted.  Every
case compares hdc_plan(..., HDC_R32 / HDC_R64) / hdc_convolve with the oracle's
real FP64 direct sum of eq. (5) element by element."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu

CFG = 700
TOLR = {"r64": 1e-12, "r32": 2e-6}
NPR = {"r64": np.float64, "r32": np.float32}


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _ops(L, C, dtype, idx):
    sh = (L,) if C == 1 else (L, C)
    return synth.uniform_real(sh, CFG, idx, 0, NPR[dtype]), synth.uniform_real(sh, CFG, idx, 1, NPR[dtype])


def _conv(L, M, m, D=0, C=1, dtype="r64", idx=0, same=False, p=0, q=0):
    import paper_2306_10016_amd as hdc
    say(f"real L={L} M={M} m={m} p={p} q={q} D={D} C={C} {dtype} same={same}")
    plan = hdc.Plan(L, M, m, p, q, C, D, dtype)
    f, g = _ops(L, C, dtype, idx)
    if same:
        g = f
    ft = to_dev(f)
    gt = ft if same else to_dev(g)
    h = _host(plan.convolve(ft, gt))
    return plan, f.astype(np.float64), g.astype(np.float64), h


FUSED = [
    # (L, M, m, D, C)
    (1024, 2047, 256, 1, 1),   # the small workload's shape: q = 8
    (6, 11, 4, 0, 1),          # Fig. 2's shape: p = 2, q = 3
    (37, 80, 8, 0, 1),         # M beyond 2L - 1, q = 10
    (100, 199, 16, 0, 1),      # odd q = 13 (no self-paired r = q/2)
    (1000, 1999, 64, 0, 3),    # copies
    (300, 599, 1024, 0, 1),    # q = 1: explicit padding
    (300, 599, 512, 0, 1),     # q = 2: r = 1 is its own partner
    (1, 1, 1, 0, 1),
    (500, 999, 2, 0, 1),       # m = 2, q = 500
    (777, 777, 128, 0, 2),     # first outputs (M = L)
]

ROWCOL = [
    (8192, 16383, 4096, 0, 1),      # column stage trivial (m1 = 1), q = 4
    (16384, 32767, 16384, 0, 1),    # q = 2, m1 = 4
    (10000, 19999, 8192, 0, 1),     # q = 3: residue 1 paired with 2
    (50000, 99999, 8192, 3, 1),     # p = 7, q = 13, groups of 3 with partners
    (20000, 39999, 16384, 1, 2),    # one residue per pass, copies
    (1 << 18, (1 << 19) - 1, 1 << 16, 0, 1),  # q = 8, m1 = 16
    (70000, 139999, 65536, 2, 1),   # p = 2, q = 3
    (30000, 30000, 8192, 0, 1),     # first outputs (M = L)
    (40000, 90000, 32768, 2, 3),    # M beyond 2L - 1 with copies and groups
]


@pytest.mark.parametrize("dtype", ["r64", "r32"])
@pytest.mark.parametrize("case", FUSED + ROWCOL, ids=[f"L{c[0]}_M{c[1]}_m{c[2]}_D{c[3]}_C{c[4]}" for c in FUSED + ROWCOL])
def test_real_matches_direct_sum(case, dtype):
    L, M, m, D, C = case
    plan, f, g, h = _conv(L, M, m, D, C, dtype, idx=(FUSED + ROWCOL).index(case))
    ref = oracle.direct_1d_real(f, g, M)
    err = rel(h.reshape(ref.shape), ref)
    say(f"  variant={plan.axes[0]['variant']} q={plan.axes[0]['q']} err={err:.3e}")
    assert (plan.axes[0]["variant"] == 0) == (case in FUSED)
    assert err < TOLR[dtype]


@pytest.mark.parametrize("dtype", ["r64", "r32"])
@pytest.mark.parametrize("L,m", [(1000, 256), (12000, 8192)])
def test_real_autoconvolution(L, m, dtype):
    plan, f, g, h = _conv(L, 2 * L - 1, m, dtype=dtype, idx=50 + L % 7, same=True)
    assert rel(h, oracle.direct_1d_real(f, f, 2 * L - 1)) < TOLR[dtype]


def test_real_integers_exact():
    """Integer-valued inputs round to the exact convolution (float64)."""
    import paper_2306_10016_amd as hdc
    L = 4096
    f = synth.integers_real(L, 16, CFG, 60, 0)
    g = synth.integers_real(L, 16, CFG, 60, 1)
    exact = oracle.direct_1d_real(f, g, 2 * L - 1)
    for m in (512, 4096, 8192):
        say(f"real integer exact m={m}")
        out = _host(hdc.Plan(L, 2 * L - 1, m, dtype="r64").convolve(to_dev(f), to_dev(g)))
        assert np.array_equal(np.round(out), exact)


def test_real_equals_complex_plan_on_real_inputs():
    """The real plan and the complex plan of the same shape agree on real inputs
    (the complex one carrying zero imaginary parts), and the residue-level calls
    are refused for a real plan."""
    import torch
    import paper_2306_10016_amd as hdc
    for (L, m) in ((3000, 512), (30000, 16384)):
        say(f"real vs complex L={L} m={m}")
        f, g = _ops(L, 1, "r64", 70)
        hr = _host(hdc.Plan(L, 2 * L - 1, m, dtype="r64").convolve(to_dev(f), to_dev(g)))
        hc = hdc.Plan(L, 2 * L - 1, m, dtype="c128").convolve(to_dev(f.astype(np.complex128)),
                                                              to_dev(g.astype(np.complex128)))
        torch.cuda.synchronize()
        hc = hc.cpu().numpy()
        assert np.max(np.abs(hc.imag)) < 1e-11
        assert rel(hr, hc.real) < 1e-13
    plan = hdc.Plan(1000, 1999, 256, dtype="r64")
    with pytest.raises(hdc.HdcError) as e:
        plan.forward(to_dev(f[:1000]), torch.empty(4096, dtype=torch.complex128, device="cuda"), 0)
    assert e.value.status == 2


def test_real_bitwise_deterministic():
    import paper_2306_10016_amd as hdc
    for (L, m) in ((1024, 256), (20000, 65536)):
        say(f"real determinism L={L} m={m}")
        f, g = _ops(L, 1, "r64", 80)
        plan = hdc.Plan(L, 2 * L - 1, m, dtype="r64")
        ft, gt = to_dev(f), to_dev(g)
        a = _host(plan.convolve(ft, gt))
        b = _host(plan.convolve(ft, gt))
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["r64", "r32"])
def test_real_full_size_sampled(dtype):
    """L = 2^22, M = 2^23 - 1 on sampled outputs, for the plans the sweep uses."""
    import paper_2306_10016_amd as hdc
    L = 1 << 22
    M = 2 * L - 1
    f, g = _ops(L, 1, dtype, 90)
    f64, g64 = f.astype(np.float64), g.astype(np.float64)
    ks = np.unique(np.concatenate([np.array([0, 1, L - 1, L, M - 2, M - 1]),
                                   synth.rng(CFG, 90, 3).integers(0, M, 26)]))
    ref = oracle.direct_1d_sampled(f64.astype(np.complex128), g64.astype(np.complex128), ks).real
    ft, gt = to_dev(f), to_dev(g)
    for m in (1 << 22, 1 << 21):
        say(f"real full size L=2^22 m={m} {dtype}")
        h = _host(hdc.Plan(L, M, m, dtype=dtype).convolve(ft, gt))
        err = rel(h[ks], ref)
        say(f"   rel(sampled)={err:.3e}")
        assert err <= TOLR[dtype]
