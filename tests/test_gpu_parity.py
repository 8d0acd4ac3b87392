"""GPU parity: the HIP path (through the C-ABI) against the CPU FP64 oracle.

Bars (relative L2 over all outputs): 1e-12 for complex128, 2e-6 for
complex64; the oracle receives the complex64-rounded inputs widened to FP64.
Integer-valued inputs must round to the exact convolution in complex128.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, conv1d, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")


def _check(L, M, m, p=0, q=0, C=1, D=0, dtype="c128", cfg=200, idx=0, same=False):
    say(f"case L={L} M={M} m={m} p={p} q={q} C={C} D={D} {dtype} same={same}")
    shape = L if C == 1 else (L, C)
    f, g, f64, g64 = inputs(shape, cfg, idx, dtype)
    if same:
        g, g64 = f, f64
    plan = hdc.Plan(L, M, m, p, q, C, D, dtype)
    ft = to_dev(f)
    gt = ft if same else to_dev(g)
    h = to_host(plan.convolve(ft, gt))
    ref = oracle.padded_1d(f64, g64, M)
    err = rel(h, ref)
    say(f"   variant={plan.axes[0]['variant']} m1={plan.axes[0]['m1']} rel={err:.3e}")
    assert err <= TOL[dtype], err
    return plan, h


# -- the small workload: L=1024, M=2047, m=256, p=4, q=8, C=1, D=1, complex128
@pytest.mark.parametrize("D", [1, 3, 8])
def test_small_workload(D):
    plan, _ = _check(1024, 2047, 256, 4, 8, 1, D, "c128", cfg=1, idx=0)
    assert plan.axes[0]["variant"] == 0


@pytest.mark.parametrize("name", ["fig2_L6_M11.txt", "int_L37_M80.txt"])
def test_golden_integer_fixtures(name):
    from golden_io import load
    L, M, f, g, h = load(name)
    for m in (1, 2, 4, 8, 64):
        say(f"golden {name} m={m}")
        plan = hdc.Plan(L, M, m, dtype="c128")
        out = to_host(plan.convolve(to_dev(f), to_dev(g)))
        assert np.array_equal(np.round(out), h)
        assert rel(out, h) < 1e-13


SWEEP = []
for L in (1, 2, 3, 6, 37, 100, 513):
    for extra in (0, 7):
        M = 2 * L - 1 + extra
        # powers of two, and m = R 2^k with R in 3, 5, 7 (the mixed-radix fused kernel)
        for m in (1, 2, 4, 8, 32, 128, 1024, 3, 5, 6, 7, 12, 96, 320, 448):
            if m > 2 * M:
                continue
            SWEEP.append((L, M, m))


@pytest.mark.parametrize("L,M,m", SWEEP)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_parameter_invariance(L, M, m, dtype):
    """Every admissible (m, p, q, D) yields the same linear convolution."""
    d = hdc.derive(L, M, m, dtype=dtype)
    for D in sorted({1, 2, d["q"]}):
        if D > d["q"]:
            continue
        _check(L, M, m, 0, 0, 1, D, dtype, cfg=201, idx=L)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_nonminimal_p_q(dtype):
    """p and q above their ceilings are admissible too (q >= p, pm >= L, qm >= M)."""
    _check(100, 199, 16, 8, 14, 1, 0, dtype, cfg=202, idx=0)
    _check(100, 199, 16, 10, 20, 1, 3, dtype, cfg=202, idx=1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m,D", [(3000, 256, 0), (3000, 256, 5), (5000, 8192, 0), (5000, 8192, 1),
                                   (9000, 16384, 0), (20000, 4096, 3), (20000, 65536, 1), (777, 64, 0)])
def test_column_row_passes(L, m, D, dtype):
    M = 2 * L - 1
    d = hdc.derive(L, M, m, D=D, dtype=dtype)
    plan, _ = _check(L, M, m, 0, 0, 1, D, dtype, cfg=203, idx=L)
    if d["N"] * (16 if dtype == "c128" else 8) > 65536:
        assert plan.axes[0]["variant"] != 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,C,m", [(100, 4, 64), (37, 3, 8), (3000, 3, 8192), (2000, 5, 512),
                                   (20000, 3, 8192)])  # copies through the column/row path with p = 3
def test_copies(L, C, m, dtype):
    _check(L, 2 * L - 1, m, 0, 0, C, 0, dtype, cfg=204, idx=L)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,m", [(1000, 256), (6000, 8192)])
def test_autoconvolution(L, m, dtype):
    _check(L, 2 * L - 1, m, dtype=dtype, cfg=205, idx=L, same=True)


def test_gaussian_integers_exact():
    L = 4096
    f = synth.gaussian_integers(L, 8, 206, 0, 0)
    g = synth.gaussian_integers(L, 8, 206, 0, 1)
    exact = oracle.direct_1d(f, g, 2 * L - 1)
    for m in (512, 4096, 8192):
        say(f"integer exact m={m}")
        out = to_host(hdc.Plan(L, 2 * L - 1, m, dtype="c128").convolve(to_dev(f), to_dev(g)))
        assert np.array_equal(np.round(out), exact)


def test_bitwise_deterministic():
    for (L, m) in ((1024, 256), (20000, 65536)):
        say(f"determinism L={L} m={m}")
        f, g, _, _ = inputs(L, 207, L, "c128")
        plan = hdc.Plan(L, 2 * L - 1, m, dtype="c128")
        ft, gt = to_dev(f), to_dev(g)
        a = to_host(plan.convolve(ft, gt))
        b = to_host(plan.convolve(ft, gt))
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,M,m,D,C", [(6, 11, 4, 1, 1), (100, 199, 32, 3, 1), (1000, 2047, 256, 8, 1),
                                       (5000, 9999, 8192, 1, 1), (300, 599, 64, 2, 3)])
def test_forward_multiply_backward(L, M, m, D, C, dtype):
    """Residues equal the zero-extended N-point DFT (eq. (3)); the group loop gives h."""
    import torch
    say(f"fwd/bwd L={L} M={M} m={m} D={D} C={C} {dtype}")
    shape = L if C == 1 else (L, C)
    f, g, f64, g64 = inputs(shape, 208, L, dtype)
    plan = hdc.Plan(L, M, m, 0, 0, C, D, dtype)
    ax = plan.axes[0]
    q, N, Dg = ax["q"], ax["N"], ax["D"]
    ft, gt = to_dev(f), to_dev(g)
    Fd, Gd = plan.residue_buffer(), plan.residue_buffer()
    h = torch.empty(plan.out_shape(), dtype=ft.dtype, device="cuda")
    f2 = f64.reshape(L, C)
    Xf = np.stack([oracle.padded_dft(f2[:, c], N) for c in range(C)], axis=1)  # (N, C)
    for r0 in range(0, q, Dg):
        plan.forward(ft, Fd, r0)
        nat = to_host(plan.residues_natural(Fd, r0)).reshape(Dg, m, C)
        for d in range(min(Dg, q - r0)):
            want = Xf[q * np.arange(m) + r0 + d, :]
            assert rel(nat[d], want) <= TOL[dtype] * 4, (r0, d)
        plan.forward(gt, Gd, r0)
        plan.multiply(Fd, Gd, r0)
        plan.backward(Fd, h, r0)
    out = to_host(h)
    ref = oracle.padded_1d(f64, g64, M)
    assert rel(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_sampled(dtype):
    """L = 2^22, M = 2^23-1 (the largest sweep size) on sampled outputs."""
    L = 1 << 22
    M = 2 * L - 1
    f, g, f64, g64 = inputs(L, 209, 0, dtype)
    ks = np.unique(np.concatenate([np.array([0, 1, L - 1, L, M - 2, M - 1]),
                                   synth.rng(209, 0, 3).integers(0, M, 26)]))
    ref = oracle.direct_1d_sampled(f64, g64, ks)
    for m in (1 << 22, 1 << 21, 1 << 20):
        say(f"full size L=2^22 m={m} {dtype}")
        plan = hdc.Plan(L, M, m, dtype=dtype)
        h = to_host(plan.convolve(to_dev(f), to_dev(g)))
        err = rel(h[ks], ref)
        say(f"   rel(sampled)={err:.3e}")
        assert err <= TOL[dtype]
