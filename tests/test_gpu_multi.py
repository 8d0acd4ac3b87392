"""GPU parity of the multi-convolution (section 6.1: the convolution of A sequences):
every residue of every operand as in eq. (3), the A residues multiplied pointwise,
one backward.  Each case compares hdc_plan_multi / hdc_convolve_multi with the
oracle (the defining sum applied operand by operand, or explicit padding for the
larger cases, the two pinned to each other on the CPU)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, NP_DT, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CFG = 800


def _ops(A, L, C, dtype, idx):
    sh = (L,) if C == 1 else (L, C)
    return [synth.uniform_complex(sh, CFG, idx, w, NP_DT[dtype]) for w in range(A)]


CASES = [
    # (A, L, M, m, D, C)
    (3, 100, None, 64, 0, 1),          # fused, q = 5
    (4, 37, None, 16, 0, 1),           # fused, q = 9
    (8, 20, None, 32, 2, 1),           # eight operands
    (3, 1000, None, 4096, 0, 1),       # q = 1: explicit padding
    (3, 500, 700, 256, 0, 1),          # first outputs (M below 3(L-1)+1)
    (5, 64, None, 64, 0, 2),           # copies
    (2, 3000, None, 512, 0, 1),        # two operands through the multi entry point
    (3, 20000, None, 16384, 0, 1),     # column/row/column, q = 4, m1 = 4
    (4, 50000, None, 65536, 2, 1),     # q = 4 in groups of 2
    (3, 1 << 18, None, 1 << 18, 1, 1),  # q = 3, one residue per pass, m1 = 64
    (6, 4000, None, 8192, 0, 3),       # copies, q = 3
    (3, 9000, 12000, 8192, 0, 1),      # first outputs, column/row/column
]


def _ref(xs, A, L, M):
    M = A * (L - 1) + 1 if M is None else M
    if L * L * (A - 1) <= 5e8:
        return oracle.direct_multi([x.astype(np.complex128) for x in xs], M)
    return oracle.padded_multi([x.astype(np.complex128) for x in xs], M)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", CASES, ids=[f"A{c[0]}_L{c[1]}_M{c[2]}_m{c[3]}_D{c[4]}_C{c[5]}" for c in CASES])
def test_multi_matches_oracle(case, dtype):
    import paper_2306_10016_amd as hdc
    A, L, M, m, D, C = case
    say(f"multi A={A} L={L} M={M} m={m} D={D} C={C} {dtype}")
    plan = hdc.MultiPlan(A, L, M, m=m, C=C, D=D, dtype=dtype)
    xs = _ops(A, L, C, dtype, CASES.index(case))
    h = to_host(plan.convolve([to_dev(x) for x in xs]))
    ref = _ref(xs, A, L, M)
    err = rel(h.reshape(ref.shape), ref)
    say(f"  q={plan.axes[0]['q']} variant={plan.axes[0]['variant']} err={err:.3e}")
    assert plan.axes[0]["N"] >= max(plan.axes[0]["M"], A * (L - 1) + 1)
    assert err < TOL[dtype]


def test_multi_integers_exact_and_residue_level():
    """Gaussian-integer operands round to the exact result; the residue-level calls
    (forward of each operand, products, backward) give the same convolution."""
    import torch
    import paper_2306_10016_amd as hdc
    A, L = 3, 3000
    xs = [synth.gaussian_integers(L, 4, CFG, 40, w) for w in range(A)]
    exact = oracle.direct_multi(xs, A * (L - 1) + 1)
    for m in (1024, 4096, 8192):
        plan = hdc.MultiPlan(A, L, m=m, dtype="c128")
        out = to_host(plan.convolve([to_dev(x) for x in xs]))
        say(f"multi integer exact m={m}")
        assert np.array_equal(np.round(out), exact)
    plan = hdc.MultiPlan(A, L, m=1024, D=2, dtype="c128")
    ax = plan.axes[0]
    xd = [to_dev(x) for x in xs]
    bufs = [plan.residue_buffer() for _ in range(A)]
    h = torch.empty(plan.out_shape(), dtype=torch.complex128, device="cuda")
    for r0 in range(0, ax["q"], ax["D"]):
        for x, b in zip(xd, bufs):
            plan.forward(x, b, r0)
        for b in bufs[1:]:
            plan.multiply(bufs[0], b, r0)
        plan.backward(bufs[0], h, r0)
    assert np.array_equal(np.round(to_host(h)), exact)
    with pytest.raises(hdc.HdcError) as e:
        plan.__class__.__mro__[1].convolve(plan, xd[0], xd[1])
    assert e.value.status == 1


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_multi_full_size_sampled(dtype):
    """Three operands of 2^20 points (transform 2^22 > 3 L) on sampled outputs."""
    import paper_2306_10016_amd as hdc
    A, L = 3, 1 << 20
    K = A * (L - 1) + 1
    xs = _ops(A, L, 1, dtype, 50)
    ks = np.unique(np.concatenate([np.array([0, 1, L, K // 2, K - 2, K - 1]),
                                   synth.rng(CFG, 50, 3).integers(0, K, 20)]))
    ref = oracle.multi_sampled([x.astype(np.complex128) for x in xs], ks)
    xd = [to_dev(x) for x in xs]
    for m in (1 << 22, 1 << 20):
        say(f"multi full size A=3 L=2^20 m={m} {dtype}")
        h = to_host(hdc.MultiPlan(A, L, m=m, dtype=dtype).convolve(xd))
        err = rel(h[ks], ref)
        say(f"   rel(sampled)={err:.3e}")
        assert err <= TOL[dtype]
