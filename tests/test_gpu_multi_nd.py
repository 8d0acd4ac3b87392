"""2D/3D multi-convolution (section 6.1 applied axis by axis, section 3.6):
h = x_0 * ... * x_{A-1} for A = 3 .. 5 boxes, against the oracle's padded N-D
convolution applied operand by operand.  Both dtypes; the innermost axis on the
fused kernel and on the column/row/column passes; an outer axis split in two
column stages (m = 2048); residue groups (D < q); first outputs (M below the
A(L-1)+1 terms); A = 2 through the multi entry point equal to hdc_convolve of
an N-D plan; exact Gaussian-integer results."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import NP_DT, TOL, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")


def _ref(xs, M):
    """The A-fold linear convolution (every term), then its first M per axis."""
    acc = xs[0].astype(np.complex128)
    for x in xs[1:]:
        full = tuple(a + b - 1 for a, b in zip(acc.shape, x.shape))
        acc = oracle.padded_nd(acc, x.astype(np.complex128), full)
    return acc[tuple(slice(0, k) for k in M)]


def _operands(A, L, dtype, cfg):
    return [synth.uniform_complex(tuple(L), cfg, sum(L), o, NP_DT[dtype]) for o in range(A)]


# (A, L, M, m, D)
CASES = [
    (3, (20, 30), None, None, None),
    (3, (33, 100), None, (64, 128), None),
    (4, (10, 12, 14), None, None, None),
    (3, (300, 1500), None, (512, 2048), None),     # inner q = 3: fused in c64, column/row/column in c128
    (5, (16, 700), None, (16, 1024), None),
    (3, (40, 50), (60, 70), None, None),           # first outputs on both axes
    (3, (1500, 20), None, (2048, 32), None),       # outer m = 1024 x 2: two column stages
    (3, (40, 60), None, (64, 64), (1, 2)),         # residue groups on both axes
    (3, (6, 9, 300), None, (8, 16, 512), (0, 2, 0)),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("A,L,M,m,D", CASES)
def test_multi_nd_against_oracle(A, L, M, m, D, dtype):
    plan = hdc.MultiPlan.nd(A, L, M, m, D, dtype=dtype)
    Mo = tuple(ax["M"] for ax in plan.axes)
    say(f"multi nd A={A} L={L} M={Mo} m={[ax['m'] for ax in plan.axes]} q={[ax['q'] for ax in plan.axes]} "
        f"variants={[ax['variant'] for ax in plan.axes]} {dtype}")
    xs = _operands(A, L, dtype, 970)
    h = to_host(plan.convolve([to_dev(x) for x in xs]))
    ref = _ref(xs, Mo)
    err = rel(h, ref)
    say(f"   rel={err:.3e}")
    assert err <= TOL[dtype], err


def test_inner_axis_paths_differ_by_dtype():
    p64 = hdc.MultiPlan.nd(3, (300, 1500), None, (512, 2048), dtype="c64")
    p128 = hdc.MultiPlan.nd(3, (300, 1500), None, (512, 2048), dtype="c128")
    assert p64.axes[1]["variant"] == 0 and p128.axes[1]["variant"] == 1


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_operands_equal_hdc_convolve(dtype):
    L = (50, 70)
    xs = _operands(2, L, dtype, 971)
    mp = hdc.MultiPlan.nd(2, L, dtype=dtype)
    a = to_host(mp.convolve([to_dev(x) for x in xs]))
    plan = hdc.Plan.nd(list(L), [2 * x - 1 for x in L], [ax["m"] for ax in mp.axes], dtype=dtype)
    b = to_host(plan.convolve(to_dev(xs[0]), to_dev(xs[1])))
    assert rel(a, b) <= TOL[dtype]
    assert rel(a, _ref(xs, tuple(2 * x - 1 for x in L))) <= TOL[dtype]


def test_gaussian_integers_exact():
    A, L = 3, (12, 17)
    xs = [synth.gaussian_integers(L, 6, 972, 0, o) for o in range(A)]
    plan = hdc.MultiPlan.nd(A, L, dtype="c128")
    out = to_host(plan.convolve([to_dev(x) for x in xs]))
    exact = _ref(xs, tuple(A * (x - 1) + 1 for x in L))
    assert np.array_equal(np.round(out), np.round(exact))


def test_refuses_bad_arguments():
    with pytest.raises(hdc.HdcError):
        hdc.MultiPlan.nd(9, (10, 10))             # more than 8 operands
    with pytest.raises(hdc.HdcError):
        hdc.MultiPlan.nd(3, (10, 10), m=(16, 12))  # m not a power of two
