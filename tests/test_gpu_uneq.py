"""GPU parity of the unequal-length convolution (section 3.5): the shorter
operand in m-point residues, the longer in Lambda m-point ones, matched by
r_f = q_g lambda + r_g.  Every case compares hdc_plan_uneq / hdc_convolve with
the FP64 oracle's direct sum of eq. (5) element by element."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, NP_DT, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CFG = 600


def _ops(Lf, Lg, C, dtype, idx):
    shf = (Lf,) if C == 1 else (Lf, C)
    shg = (Lg,) if C == 1 else (Lg, C)
    f = synth.uniform_complex(shf, CFG, idx, 0, NP_DT[dtype])
    g = synth.uniform_complex(shg, CFG, idx, 1, NP_DT[dtype])
    return f, g


def _run(Lf, Lg, M=None, m=0, lam=0, C=1, D=0, dtype="c128", idx=0):
    import paper_2306_10016_amd as hdc
    M = Lf + Lg - 1 if M is None else M
    say(f"uneq Lf={Lf} Lg={Lg} M={M} m={m} lam={lam} C={C} D={D} {dtype}")
    plan = hdc.UneqPlan(Lf, Lg, M, m=m, lam=lam, C=C, D=D, dtype=dtype)
    f, g = _ops(Lf, Lg, C, dtype, idx)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    return plan, f, g, h


SMALL = [
    # (Lf, Lg, m, lam, D, C)
    (12, 1000, 0, 0, 0, 1),
    (12, 1000, 16, 4, 0, 1),
    (12, 1000, 16, 4, 3, 1),
    (2, 777, 8, 8, 1, 1),
    (1, 500, 1, 64, 0, 1),
    (37, 38, 8, 2, 2, 1),
    (100, 2187, 32, 16, 5, 1),
    (100, 2187, 128, 1, 0, 1),      # Lambda = 1: same m, different lengths (single fused kernel)
    (300, 1000, 256, 1, 0, 2),      # Lambda = 1 fused with copies and p_f > 1
    (700, 6000, 2048, 1, 2, 1),     # Lambda = 1 too large to fuse: row pass with the raw operand
    (300, 5000, 64, 32, 0, 3),      # copies
    (513, 4097, 256, 16, 2, 2),
    (1000, 100000, 1024, 16, 0, 1),  # p_g > 1
    (1000, 100000, 32768, 4, 0, 1),  # the shorter operand's column stage m1f = 8
    (5, 20000, 4, 1024, 0, 1),       # Lambda at the column-stage limit
    (4096, 70000, 8192, 16, 3, 1),   # m1f = 2 with residue groups
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", SMALL, ids=[f"Lf{c[0]}_Lg{c[1]}_m{c[2]}_lam{c[3]}_D{c[4]}_C{c[5]}" for c in SMALL])
def test_uneq_matches_direct_sum(case, dtype):
    Lf, Lg, m, lam, D, C = case
    plan, f, g, h = _run(Lf, Lg, m=m, lam=lam, C=C, D=D, dtype=dtype, idx=SMALL.index(case))
    ref = oracle.direct_1d(f.astype(np.complex128), g.astype(np.complex128), Lf + Lg - 1)
    err = rel(h.reshape(ref.shape), ref)
    say(f"  axes long={plan.axes[0]} short={plan.short_axis} err={err:.3e}")
    assert err < TOL[dtype]


def test_uneq_swapped_roles_and_longer_output():
    """f longer than g (roles swap) and M beyond Lf + Lg - 1 (zeros there)."""
    plan, f, g, h = _run(3000, 40, M=3100, m=64, lam=8, idx=20)
    assert plan.short_axis["L"] == 40 and plan.axes[0]["L"] == 3000
    ref = oracle.direct_1d(f, g, 3100)
    assert rel(h, ref) < TOL["c128"]
    assert np.all(np.abs(h[3039:]) < 1e-13)


def test_uneq_equal_lengths_lambda():
    """Equal lengths through the unequal plan with Lambda > 1."""
    plan, f, g, h = _run(640, 640, m=64, lam=4, idx=21)
    assert rel(h, oracle.direct_1d(f, g, 1279)) < TOL["c128"]


def test_uneq_integer_exact():
    """Gaussian integers: every product and sum is exact in FP64."""
    import paper_2306_10016_amd as hdc
    Lf, Lg = 12, 4000
    f = synth.gaussian_integers(Lf, 16, CFG, 30, 0)
    g = synth.gaussian_integers(Lg, 16, CFG, 30, 1)
    plan = hdc.UneqPlan(Lf, Lg, m=16, lam=16)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert np.array_equal(np.round(h), oracle.direct_1d(f, g, Lf + Lg - 1))


@pytest.mark.parametrize("lam", [1, 4, 32])
def test_uneq_matched_residues(lam):
    """hdc_forward_operand: the shorter operand's m-point residues, matched into the
    longer operand's geometry, hold the length-N transform at k = q_g l_g + r_g;
    so do the longer operand's own residues."""
    import torch
    import paper_2306_10016_amd as hdc
    Lf, Lg = 50, 3000
    plan = hdc.UneqPlan(Lf, Lg, m=64, lam=lam, D=2)
    f, g = _ops(Lf, Lg, 1, "c128", 40 + lam)
    G = plan.axes[0]
    qg, mg, N = G["q"], G["m"], G["N"]
    Ff = oracle.padded_dft(f, N)
    Fg = oracle.padded_dft(g, N)
    say(f"matched residues lam={lam} long={G} short={plan.short_axis}")
    for r0 in range(0, qg, 2):
        Dg = min(2, qg - r0)
        for op, x, ref in ((0, f, Ff), (1, g, Fg)):
            buf = plan.residue_buffer()
            plan.forward_operand(op, to_dev(x), buf, r0)
            nat = to_host(plan.residues_natural(buf, r0))[: Dg * mg].reshape(Dg, mg)
            for d in range(Dg):
                want = ref[qg * np.arange(mg) + r0 + d]
                assert rel(nat[d], want) < 1e-12, (op, r0, d)


def test_uneq_residue_level_path_matches_convolve():
    """forward_operand (both operands), multiply and backward per group give the convolution."""
    import paper_2306_10016_amd as hdc
    import torch
    Lf, Lg = 20, 2500
    plan = hdc.UneqPlan(Lf, Lg, m=32, lam=8, D=2)
    f, g = _ops(Lf, Lg, 1, "c128", 50)
    fd, gd = to_dev(f), to_dev(g)
    h = torch.empty(Lf + Lg - 1, dtype=torch.complex128, device="cuda")
    for r0 in range(0, plan.axes[0]["q"], 2):
        F = plan.residue_buffer()
        Gb = plan.residue_buffer()
        plan.forward_operand(0, fd, F, r0)
        plan.forward_operand(1, gd, Gb, r0)
        plan.multiply(F, Gb, r0)
        plan.backward(F, h, r0)
    assert rel(to_host(h), oracle.direct_1d(f, g, Lf + Lg - 1)) < TOL["c128"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_uneq_full_size_sampled(dtype):
    """A short filter against a 2^22-point signal at the largest Lambda m, checked
    at sampled outputs (both ends, the block edges, random interior points)."""
    Lf, Lg = 12, 1 << 22
    plan, f, g, h = _run(Lf, Lg, m=4096, lam=1024, dtype=dtype, idx=60)
    mg = plan.axes[0]["m"]
    r = synth.rng(CFG, 61, 0)
    K = Lf + Lg - 1
    ks = np.unique(np.concatenate([np.arange(16), K - 16 + np.arange(16), [mg - 1, mg, mg + 1, K // 2],
                                   r.integers(0, K, 400)]))
    ref = oracle.direct_1d_sampled(f.astype(np.complex128), g.astype(np.complex128), ks)
    err = rel(h[ks], ref)
    say(f"  full size err={err:.3e}")
    assert err < TOL[dtype]


def test_uneq_deterministic():
    plan, f, g, h1 = _run(12, 50000, m=64, lam=64, idx=70)
    h2 = to_host(plan.convolve(to_dev(f), to_dev(g)))
    assert np.array_equal(h1, h2)


@pytest.mark.parametrize("case,path", [((100, 2187, 128, 1, 0, 1), "fused"), ((700, 6000, 2048, 1, 2, 1), "raw"),
                                       ((12, 1000, 16, 4, 0, 1), "raw"), ((1000, 100000, 32768, 4, 0, 1), "general")])
def test_uneq_execution_paths(case, path):
    """Which kernels run: one fused kernel (Lambda = 1 and the transform fits a
    workgroup), the row pass forming the shorter operand from its input (its
    column stage trivial), or both column stages; the workspace follows."""
    import paper_2306_10016_amd as hdc
    Lf, Lg, m, lam, D, C = case
    plan = hdc.UneqPlan(Lf, Lg, m=m, lam=lam, C=C, D=D)
    G = plan.axes[0]
    one = min(G["D"], G["q"]) * G["m"] * C * 16
    want = {"fused": 0, "raw": one, "general": 2 * one}[path]
    assert plan.workspace_bytes == want
    f, g = _ops(Lf, Lg, C, "c128", 80)
    fd, gd = to_dev(f), to_dev(g)
    out = to_dev(np.zeros(Lf + Lg - 1, np.complex128))
    kinds = [k for k, _, _ in plan.convolve_profiled(fd, gd, out)]
    groups = -(-G["q"] // min(G["D"], G["q"]))
    per = {"fused": ["fused"], "raw": ["col_fwd", "row", "col_bwd"],
           "general": ["col_fwd", "col_fwd", "row", "col_bwd"]}[path]
    assert kinds == ([] if path == "fused" else []) + per * (1 if path == "fused" else groups)
    assert rel(to_host(out), oracle.direct_1d(f, g, Lf + Lg - 1)) < TOL["c128"]
