"""Real data in 2D and 3D (the real case of section 7): h = Im(z * z) / (2 s) for
z = f + i s g, one complex autoconvolution with s = max|f| / max|g| (z formed
and h extracted inside the outer axis's column passes).  Against the oracle's padded N-D convolution of the same (real-valued)
data in float64 and float32: the innermost axis on the fused kernel, the
row-convolution kernel (float32) and the column/row/column passes; an outer
axis split in two column stages; 3D; first outputs; operands whose scales
differ by 10^6 (the scale s keeps the error relative to |f| |g| at a complex
plan's); g = 0 (rounding noise at the scale of f * f); autoconvolution (f = g);
integer-valued data exact in float64; bitwise replay."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, rel, say, to_dev

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")

NP_R = {"r64": np.float64, "r32": np.float32}
TOL_R = {"r64": TOL["c128"], "r32": TOL["c64"]}


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _ref(f, g, M):
    L = f.shape
    K = tuple(max(mm, 2 * a - 1) for mm, a in zip(M, L))
    full = oracle.padded_nd(f.astype(np.complex128), g.astype(np.complex128), K)
    return full[tuple(slice(0, k) for k in M)].real


def _inputs(L, cfg, dtype, gscale=1.0):
    r = synth.rng(cfg, sum(L), 0)
    f = r.uniform(-1, 1, L).astype(NP_R[dtype])
    g = (gscale * r.uniform(-1, 1, L)).astype(NP_R[dtype])
    return f, g


# (L, M, m)
CASES = [
    ((20, 30), None, None),
    ((33, 700), None, (64, 1024)),
    ((300, 1500), None, (512, 2048)),
    ((1500, 40), None, (2048, 64)),               # outer m = 1024 x 2
    ((3000, 20), None, (2048, 32)),               # outer m = 1024 x 2, q = 3 residues in one group
    ((6, 9, 300), None, (8, 16, 512)),
    ((40, 50), (60, 70), None),                    # first outputs
    ((16, 3000), None, (16, 4096)),                # inner axis: row convolution in float32
]


def _plan(L, M, m, dtype):
    M = tuple(2 * a - 1 for a in L) if M is None else M
    m = tuple(1 << (a - 1).bit_length() for a in L) if m is None else m
    return hdc.Plan.nd(list(L), list(M), list(m), dtype=dtype), M


@pytest.mark.parametrize("dtype", ["r64", "r32"])
@pytest.mark.parametrize("L,M,m", CASES)
def test_real_nd_against_oracle(L, M, m, dtype):
    plan, M = _plan(L, M, m, dtype)
    say(f"real nd L={L} M={M} m={[a['m'] for a in plan.axes]} variants={[a['variant'] for a in plan.axes]} {dtype}")
    f, g = _inputs(L, 980, dtype)
    h = _host(plan.convolve(to_dev(f), to_dev(g)))
    err = rel(h, _ref(f, g, M))
    say(f"   rel={err:.3e}")
    assert h.shape == tuple(M) and err <= TOL_R[dtype], err


@pytest.mark.parametrize("dtype", ["r64", "r32"])
def test_unbalanced_scales_and_zero(dtype):
    L = (40, 300)
    plan, M = _plan(L, None, None, dtype)
    for gs in (1e-6, 1e6):
        f, g = _inputs(L, 981, dtype, gscale=gs)
        h = _host(plan.convolve(to_dev(f), to_dev(g)))
        err = rel(h, _ref(f, g, M))
        say(f"   g scale {gs:g}: rel={err:.3e}")
        assert err <= TOL_R[dtype], (gs, err)
    # g = 0: s = 1 and h is the imaginary rounding of f * f, at the bar's scale of it
    f, _ = _inputs(L, 982, dtype)
    h = _host(plan.convolve(to_dev(f), to_dev(np.zeros_like(f))))
    ff = _ref(f, f, M)
    assert np.linalg.norm(h) <= TOL_R[dtype] * np.linalg.norm(ff)


@pytest.mark.parametrize("dtype", ["r64", "r32"])
def test_autoconvolution_and_replay(dtype):
    L = (50, 400)
    plan, M = _plan(L, None, None, dtype)
    f, _ = _inputs(L, 983, dtype)
    ft = to_dev(f)
    a = _host(plan.convolve(ft, ft))
    b = _host(plan.convolve(ft, ft))
    assert np.array_equal(a, b)
    assert rel(a, _ref(f, f, M)) <= TOL_R[dtype]


def test_integer_valued_exact():
    L = (30, 70)
    r = synth.rng(984, 0, 0)
    f = r.integers(-8, 9, L).astype(np.float64)
    g = r.integers(-8, 9, L).astype(np.float64)
    plan, M = _plan(L, None, None, "r64")
    h = _host(plan.convolve(to_dev(f), to_dev(g)))
    exact = oracle.direct_nd_sampled(f.astype(np.complex128), g.astype(np.complex128), M,
                                     np.arange(int(np.prod(M)))).real.reshape(M)
    assert np.array_equal(np.round(h), np.round(exact))


def test_one_dimensional_real_data_take_the_1d_plan():
    with pytest.raises(hdc.HdcError):
        hdc.Plan.nd([100], [199], [128], dtype="r64")
