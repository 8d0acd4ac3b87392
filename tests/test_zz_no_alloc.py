"""hdc_convolve_noalloc: the convolution with the library's per-GPU scratch array
as its workspace (for callers that cannot allocate), against hdc_convolve with a
caller workspace on the same inputs.  Calls run back to back, each later one on a
smaller problem, so every call finds the array holding the previous call's data;
the results must equal hdc_convolve's bit for bit (same kernels, same plan)."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")


def _pair(plan, f, g):
    import torch
    ft, gt = to_dev(f), to_dev(g)
    ref = plan.convolve(ft, gt)
    out = torch.full_like(ref, complex(np.nan, np.nan))
    plan.convolve_noalloc(ft, gt, out)
    return to_host(out), to_host(ref)


# (L, M, m, D, C, dtype), largest first; the first fills the whole array
CASES_1D = [
    (1 << 20, (1 << 21) - 1, 1 << 20, 2, 1, "c128"),  # workspace 2 D m C 16 B = 64 MiB, the maximum
    (6000, 11999, 8192, 0, 1, "c128"),
    (3000, 5999, 1024, 0, 2, "c64"),
    (1024, 2047, 256, 1, 1, "c128"),                 # fused kernel: no workspace at all
]


def test_noalloc_1d_sequence_equals_convolve():
    for i, (L, M, m, D, C, dt) in enumerate(CASES_1D):
        say(f"noalloc 1D L={L} m={m} D={D} C={C} {dt}")
        plan = hdc.Plan(L, M, m, D=D, C=C, dtype=dt)
        assert plan.workspace_bytes <= hdc.SCRATCH_BYTES
        f, g, f64, g64 = inputs(L if C == 1 else (L, C), 700, i, dt)
        h, ref = _pair(plan, f, g)
        assert np.array_equal(h, ref)
        if L <= 6000:
            exact = oracle.padded_1d(f64, g64, M) if C == 1 else np.stack(
                [oracle.padded_1d(f64[:, c], g64[:, c], M) for c in range(C)], axis=1)
            assert rel(h, exact) <= TOL[dt]


def test_noalloc_other_plan_kinds():
    import torch
    # 2D, unequal lengths and real data after a large call, then a smaller call of each again
    for rnd in range(2):
        s = 1 if rnd == 0 else 2
        say(f"noalloc 2D / unequal / real, round {rnd}")
        L2 = (300 // s, 700 // s)
        plan = hdc.Plan.nd(L2, [2 * a - 1 for a in L2], [256, 1024 // s], dtype="c128")
        say(f"   2D workspace {plan.workspace_bytes} bytes")
        assert 0 < plan.workspace_bytes <= hdc.SCRATCH_BYTES
        f, g, _, _ = inputs(L2, 701, rnd, "c128")
        h, ref = _pair(plan, f, g)
        assert np.array_equal(h, ref)
        up = hdc.UneqPlan(12, 50000 // s, 50000 // s + 11, m=2048, lam=16, dtype="c128")
        assert up.workspace_bytes <= hdc.SCRATCH_BYTES
        fu, _, _, _ = inputs(12, 702, rnd, "c128")
        gu, _, _, _ = inputs(50000 // s, 703, rnd, "c128")
        a = up.convolve(to_dev(fu), to_dev(gu))
        b = torch.full_like(a, complex(np.nan, np.nan))
        up.convolve_noalloc(to_dev(fu), to_dev(gu), b)
        assert np.array_equal(to_host(a), to_host(b))
        Lr = 70000 // s
        rp = hdc.Plan(Lr, 2 * Lr - 1, 65536 // s, dtype="r64")
        assert 0 < rp.workspace_bytes <= hdc.SCRATCH_BYTES
        fr = np.random.default_rng(rnd).uniform(-1, 1, Lr)
        gr = np.random.default_rng(rnd + 9).uniform(-1, 1, Lr)
        a = rp.convolve(torch.from_numpy(fr).cuda(), torch.from_numpy(gr).cuda())
        b = torch.full_like(a, np.nan)
        rp.convolve_noalloc(torch.from_numpy(fr).cuda(), torch.from_numpy(gr).cuda(), b)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_noalloc_rejects_plans_beyond_the_array():
    import torch
    L = 1 << 22
    plan = hdc.Plan(L, 2 * L - 1, L, dtype="c128")  # workspace 2 x 2 x 2^22 x 16 B = 256 MiB
    assert plan.workspace_bytes > hdc.SCRATCH_BYTES
    f = torch.zeros(L, dtype=torch.complex128, device="cuda")
    h = torch.zeros(2 * L - 1, dtype=torch.complex128, device="cuda")
    with pytest.raises(hdc.HdcError) as e:
        plan.convolve_noalloc(f, f, h)
    assert e.value.status == 3
