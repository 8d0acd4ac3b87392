"""Whole-row convolution of an innermost N-D axis (variant 3): one workgroup per
row runs the row's residues in turn and keeps the output sums of eq. (4) in
registers (complex64; complex128 inner axes keep the other variants).  Against
the oracle's padded N-D convolution: m = 1024, 2048 and 4096, p from 1 to 4,
every number of output blocks the registers hold (up to 4), first outputs
(q_out < q), a zero tail,
a half-empty workgroup (one row, two rows per workgroup), 3D, autoconvolution
and bitwise replay."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, inputs, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")

# (L, M, m, dtype): the innermost axis takes variant 3
CASES = [
    ((1, 1500), (1, 2999), (1, 1024), "c64"),          # one row, two rows per workgroup: half empty
    ((33, 1500), (65, 2999), (64, 1024), "c64"),       # p = 2, q = 3
    ((20, 3000), (39, 5999), (32, 2048), "c64"),       # p = 2, q = 3
    ((16, 7000), (31, 13999), (16, 4096), "c64"),      # p = 2, q = 4 = q_out
    ((8, 4000), (15, 4000), (8, 1024), "c64"),         # p = 4, q = 8, first outputs: q_out = 4
    ((16, 1500), (31, 4000), (16, 1024), "c64"),       # zero tail: M beyond 2L - 1
    ((12, 900), (23, 1799), (16, 1024), "c64"),        # q = 2, one input block
    ((16, 2000), (31, 3999), (16, 2048), "c64"),       # p = 1, q = 2
    ((8, 4000), (15, 7999), (8, 4096), "c64"),         # p = 1, q = 2
    ((8, 5000), (15, 5000), (8, 4096), "c64"),         # p = 2, q = 3, first outputs: q_out = 2
    ((4, 6, 3000), (7, 11, 5999), (4, 8, 2048), "c64"),   # 3D
]


def _plan(L, M, m, dtype):
    plan = hdc.Plan.nd(list(L), list(M), list(m), dtype=dtype)
    ax = plan.axes[-1]
    assert ax["variant"] == 3, ax
    return plan


@pytest.mark.parametrize("L,M,m,dtype", CASES)
def test_rowconv_against_oracle(L, M, m, dtype):
    plan = _plan(L, M, m, dtype)
    ax = plan.axes[-1]
    say(f"rowconv L={L} M={M} m={m} {dtype} p={ax['p']} q={ax['q']} q_out={ax['q_out']}")
    f, g, f64, g64 = inputs(tuple(L), 960, sum(L), dtype)
    h = to_host(plan.convolve(to_dev(f), to_dev(g)))
    K = tuple(max(a, 2 * b - 1) for a, b in zip(M, L))
    ref = oracle.padded_nd(f64, g64, K)[tuple(slice(0, a) for a in M)]
    err = rel(h, ref)
    say(f"   rel={err:.3e}")
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("L,M,m", [((16, 3000), (31, 5999), (16, 4096)), ((8, 7000), (15, 13999), (8, 4096))])
def test_rowconv_autoconvolution_and_replay(L, M, m):
    dtype = "c64"
    plan = _plan(L, M, m, dtype)
    f, _, f64, _ = inputs(L, 961, 0, dtype)
    ft = to_dev(f)
    a = to_host(plan.convolve(ft, ft))
    b = to_host(plan.convolve(ft, ft))
    assert np.array_equal(a, b)
    assert rel(a, oracle.padded_nd(f64, f64, M)) <= TOL[dtype]


def test_complex128_keeps_the_other_variants():
    assert hdc.check_nd([16, 3000], [31, 5999], [16, 4096], dtype="c128")[-1]["variant"] != 3
