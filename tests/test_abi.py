"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol the headers declare, and hdc_derive implements the admissibility rules
of section 2.5 (p = ceil(L/m), q = ceil(M/m), pm >= L, qm >= M, q >= p)."""
import glob
import os

import pytest

import paper_2306_10016_amd as hdc
from paper_2306_10016_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_loads_and_exports_every_declared_symbol():
    L = hdc.lib()
    assert L.hdc_version().startswith(b"hdc")
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        syms = _lib.header_symbols(hdr)
        assert syms, hdr
        missing = [s for s in syms if not hasattr(L, s)]
        assert not missing, (hdr, missing)


@pytest.mark.parametrize("L,M,m,p,q", [(6, 11, 4, 2, 3), (1024, 2047, 256, 4, 8), (1, 1, 1, 1, 1),
                                       (37, 80, 64, 1, 2), (100, 199, 1, 100, 199), (1 << 22, (1 << 23) - 1,
                                                                                     1 << 22, 1, 2)])
def test_derive_ceilings(L, M, m, p, q):
    d = hdc.derive(L, M, m)
    assert (d["p"], d["q"], d["N"], d["D"]) == (p, q, p * 0 + q * m, q)
    assert d["p"] * m >= L and d["q"] * m >= M and d["q"] >= d["p"]
    assert d["q_out"] == -(-M // m)
    assert d["m1"] * d["m2"] == m


def test_derive_fig2_shape():
    """Section 2.5, Fig. 2: L=6, M=11, m=4 gives p=2 (explicit pad to 8) and q=3 (implicit to 12)."""
    d = hdc.derive(6, 11, 4)
    assert d["p"] == 2 and d["q"] == 3 and d["N"] == 12


@pytest.mark.parametrize("args,status", [
    ((10, 18, 4, 0, 4), 1),      # q m = 16 < 2L-1 = 19: the transform aliases
    ((10, 0, 4), 1),             # M < 1
    ((0, 5, 4), 1),              # L < 1
    ((10, 19, 0), 1),            # m < 1
    ((10, 19, 4, 2, 0), 1),      # p m < L
    ((10, 19, 4, 0, 4), 1),      # q m < M
    ((10, 19, 4, 5, 4), 1),      # q < p (and qm < M)
    ((10, 19, 11), 2),           # m with a prime factor above 7
    ((200, 399, 66), 2),         # m = 2 * 33: the odd factor has the prime 11
    ((10, 19, 127), 2),          # odd factor beyond 63
    ((3000, 5999, 3 * 1024), 2),  # m = 3 2^10: the residues do not fit the fused kernel's LDS
    ((10, 19, 4, 0, 0, 0), 1),   # C < 1
    ((1 << 23, (1 << 24) - 1, 1 << 24), 2),  # m beyond the column x row limit
    ((1 << 62, 1 << 40, 1 << 20), 2),           # L far beyond any supported size (2L - 1 would overflow)
    ((100, 199, 16, 1 << 62, 0), 2),            # p m would overflow
    ((100, 199, 16, 0, 1 << 61), 2),            # q m would overflow
    ((1000, 1999, 1024, 0, 0, 1 << 39), 2),     # M C beyond 2^40 (the product stays in range)
])
def test_derive_rejects(args, status):
    with pytest.raises(hdc.HdcError) as e:
        hdc.derive(*args)
    assert e.value.status == status
    assert len(str(e.value)) > 10


@pytest.mark.parametrize("m", [3, 5, 6, 7, 12, 15, 96, 320, 448, 63 * 16, 45 * 16])
def test_derive_takes_7_smooth_m(m):
    """m = R 2^k with R odd, 7-smooth and at most 63 (section 3.1's FFT-friendly
    sizes) runs on the fused kernel: variant 0."""
    L = m + 1
    d = hdc.derive(L, 2 * L - 1, m, dtype="c64")
    assert d["m"] == m and d["variant"] == 0 and d["p"] == 2 and d["q"] == 3
    # the largest: 63 sub-transforms of 64 points, q = 2 within the LDS budget
    d = hdc.derive(3000, 5999, 63 * 64, dtype="c64")
    assert d["variant"] == 0 and d["q"] == 2


def test_non_pow2_m_is_1d_complex_only():
    with pytest.raises(hdc.HdcError):
        hdc.Plan(100, 199, 12, dtype="r64")
    with pytest.raises(hdc.HdcError):
        hdc.MultiPlan(3, 100, m=12)
    with pytest.raises(hdc.HdcError):
        hdc.check_nd([100, 100], [199, 199], [16, 12])


def test_derive_clamps_D():
    assert hdc.derive(100, 199, 16, D=100)["D"] == hdc.derive(100, 199, 16)["q"]
    assert hdc.derive(100, 199, 16, D=3)["D"] == 3


def test_variant_choice_by_lds_budget():
    # the fused kernel holds q residues of m padded values (+1 slot per 8) within 80 KiB of LDS
    assert hdc.derive(1024, 2047, 256, dtype="c128")["variant"] == 0
    assert hdc.derive(4096, 8191, 4096, dtype="c128")["variant"] == 1
    assert hdc.derive(4096, 8191, 4096, dtype="c64")["variant"] == 0
    assert hdc.derive(8192, 16383, 8192, dtype="c64")["variant"] == 1
    assert hdc.derive(1 << 20, (1 << 21) - 1, 1 << 20, dtype="c64")["variant"] == 1


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises((TypeError, hdc.HdcError, RuntimeError)):
        p = hdc.Plan.__new__(hdc.Plan)
        p.dtype = 1
        hdc._check_tensor(torch.zeros(4, dtype=torch.complex128), 1, 4, "f")


def test_nd_check_is_host_only_and_reports_axes():
    d = hdc.check_nd([1024, 4096], [2047, 8191], [2048, 4096], dtype="c64")
    assert d[0]["m1"] * d[0]["m2"] == 2048 and d[0]["variant"] == 1
    assert d[1]["p"] == 1 and d[1]["q"] == 2
    with pytest.raises(hdc.HdcError):
        hdc.check_nd([1024, 4096], [2047, 8191], [1 << 21, 4096], dtype="c64")  # outer m > 2^20
    # extents whose column count (m2 x inner transform lengths) or element count
    # would leave the kernels' index ranges
    for L, m in (([1 << 20] * 3, [1 << 20, 1 << 20, 4096]), ([1 << 20, 1 << 21], [1 << 20, 1 << 22])):
        with pytest.raises(hdc.HdcError) as e:
            hdc.check_nd(L, [2 * x - 1 for x in L], m, dtype="c64")
        assert e.value.status == 2
    with pytest.raises(hdc.HdcError) as e:
        hdc.uneq_nd_check([1 << 20] * 3, [1 << 20] * 3)
    assert e.value.status == 2


@pytest.mark.parametrize("Lf,Lg,m,lam", [(12, 1000, 16, 4), (37, 38, 8, 2), (5, 20000, 4, 1024), (1000, 100000, 32768, 4),
                                         (3000, 40, 64, 8), (12, 1 << 22, 4096, 1024), (7, 9, 0, 0), (12, 1000, 0, 0)])
def test_uneq_derive_rules(Lf, Lg, m, lam):
    """Section 3.5's parameters: p_f = ceil(Ls/m), p_g = ceil(Ll/(Lambda m)),
    q_g = ceil(M/(Lambda m)), q_f = Lambda q_g, one transform length N, and the
    four-step splits that let row l1f of the shorter operand meet row
    Lambda l1f + lambda of the longer one."""
    M = Lf + Lg - 1
    s, l, sw = hdc.uneq_derive(Lf, Lg, M, m, lam)
    Ls, Ll = min(Lf, Lg), max(Lf, Lg)
    assert sw == (Lf > Lg) and s["L"] == Ls and l["L"] == Ll
    ms, ml = s["m"], l["m"]
    L_ = ml // ms
    assert ml == L_ * ms and (m == 0 or ms == m) and (lam == 0 or L_ == lam)
    assert s["p"] == -(-Ls // ms) and l["p"] == -(-Ll // ml)
    assert l["q"] == -(-M // ml) and s["q"] == L_ * l["q"]
    assert s["N"] == l["N"] == l["q"] * ml >= M
    assert l["m1"] % L_ == 0 and s["m1"] == l["m1"] // L_ and s["m2"] == l["m2"]
    assert l["m1"] * l["m2"] == ml and s["m1"] * s["m2"] == ms
    assert l["m1"] <= 1024 and l["m2"] <= 4096 and (l["variant"] == 1 or L_ == 1)
    if m == 0 and lam == 0:
        # one block up to 2^17 outputs, else the shortest transform over Lambda m with
        # at most four blocks of the longer operand; a trivial column stage for the
        # shorter one
        if M <= 131072:
            assert l["q"] == 1 and l["m"] == 1 << (M - 1).bit_length()
        else:
            Ns = [-(-M // (1 << k)) * (1 << k) for k in range(23) if 4 * (1 << k) >= Ll or k == 22]
            assert l["p"] <= 4 and l["N"] == min(Ns)
        assert s["m1"] == 1


def test_uneq_derive_errors():
    with pytest.raises(hdc.HdcError) as e:
        hdc.uneq_derive(12, 1000, 0)
    assert e.value.status == 1
    for m, lam in ((24, 2), (16, 3), (16, 2048), (8192, 1024)):
        with pytest.raises(hdc.HdcError) as e:
            hdc.uneq_derive(12, 1000, 1011, m, lam)
        assert e.value.status == 2
    with pytest.raises(hdc.HdcError):
        hdc.uneq_derive(0, 1000, 1011)
    with pytest.raises(hdc.HdcError) as e:  # Lf + Lg - 1 would overflow
        hdc.uneq_derive(1 << 62, 1 << 62, 1 << 62)
    assert e.value.status == 2


@pytest.mark.parametrize("sf,sg,m,lam", [((12, 12), (4096, 4096), None, None), ((5, 8), (3000, 20), (8, 8), (512, 4)),
                                         ((9, 3, 12), (4, 30, 5), None, None), ((100, 6), (2500, 40), (128, 8), (16, 8))])
def test_uneq_nd_check_rules(sf, sg, m, lam):
    """Per axis the 1D rules of section 3.5; outer axes split into two column stages
    of at most 1024 with Lambda dividing the first, the shorter operand's split the
    longer one's divided by Lambda."""
    res = hdc.uneq_nd_check(sf, sg, m=m, lam=lam)
    n = len(sf)
    for a, (s, l, sw) in enumerate(res):
        L_ = l["m"] // s["m"]
        assert sw == (sf[a] > sg[a]) and s["L"] == min(sf[a], sg[a]) and l["L"] == max(sf[a], sg[a])
        assert s["N"] == l["N"] >= sf[a] + sg[a] - 1 and s["q"] == L_ * l["q"]
        assert l["m1"] % L_ == 0 and s["m1"] * L_ == l["m1"] and s["m2"] == l["m2"]
        if a < n - 1:
            assert l["m1"] == max(min(l["m"], 1024), L_) and l["m2"] <= 1024 and l["variant"] == 1
        else:
            assert l["m2"] <= 4096


def test_uneq_nd_check_errors():
    with pytest.raises(hdc.HdcError):
        hdc.uneq_nd_check((4, 4), (10, 10), M=(0, 13))
    with pytest.raises(hdc.HdcError) as e:  # outer Lambda m above 2^20
        hdc.uneq_nd_check((4, 4), (3000000, 10), m=(4096, 4), lam=(512, 1))
    assert e.value.status == 2



@pytest.mark.parametrize("L,M,m", [(10, 10, 4), (1000, 1000, 256), (1000, 1, 64), (4096, 4096, 4096), (37, 50, 8)])
def test_first_outputs_mode(L, M, m):
    """M below 2L-1 (the backward range of section 2.2 gives the first L outputs):
    the transform still covers 2L-1 points, the backward writes ceil(M/m) blocks."""
    d = hdc.derive(L, M, m)
    assert d["q"] == -(-(2 * L - 1) // m) and d["N"] >= 2 * L - 1
    assert d["q_out"] == -(-M // m) and d["M"] == M


def test_uneq_first_outputs_mode():
    s, l, _ = hdc.uneq_derive(12, 1000, 500, 16, 4)
    assert l["q"] == -(-1011 // 64) and l["q_out"] == -(-500 // 64) and l["M"] == 500


def test_real_dtype_rules():
    """Real data (HDC_R32 / HDC_R64) derive exactly as the complex plan of the same
    shape, in 1D and N-D (whose real plans run the complex autoconvolution of
    z = f + i s g), and are refused, with HDC_ERR_UNSUPPORTED, by the unequal-length
    entry points."""
    for L, M, m in [(6, 11, 4), (1024, 2047, 256), (1 << 22, (1 << 23) - 1, 1 << 22)]:
        assert hdc.derive(L, M, m, dtype="r64") == hdc.derive(L, M, m, dtype="c128")
        assert hdc.derive(L, M, m, dtype="r32") == hdc.derive(L, M, m, dtype="c64")
    assert hdc.check_nd([16, 16], [31, 31], [16, 16], dtype="r64") == \
        hdc.check_nd([16, 16], [31, 31], [16, 16], dtype="c128")
    with pytest.raises(hdc.HdcError) as e:
        hdc.uneq_derive(12, 1000, 1011, dtype="r32")
    assert e.value.status == 2


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_largest_1d_geometry_fits_lds(dtype):
    """Every kernel geometry of the largest 1D plans (column stage 1024, row stage
    4096, their twiddle tables) fits the LDS of a gfx950 workgroup."""
    for L in (1 << 22, 1 << 21, 3 ** 13):
        for m in (1 << 22, 1 << 21, 1 << 20, 4096):
            if m * 2 < L:
                continue
            ax = hdc.check_nd([L], [2 * L - 1], [m], dtype=dtype)[0]
            assert ax["m1"] * ax["m2"] == m


def test_multi_plan_rejects_before_touching_the_device():
    """hdc_plan_multi validates on the host: operand count, lengths, and sizes whose
    term count A (L - 1) + 1 would overflow."""
    for args, kw, status in [((1, 100), {}, 1), ((9, 100), {}, 1), ((3, 0), {}, 1),
                             ((3, 1 << 62), {"M": 100}, 2), ((3, 100), {"m": 64, "q": 2}, 1)]:
        with pytest.raises(hdc.HdcError) as e:
            hdc.MultiPlan(*args, **kw)
        assert e.value.status == status, (args, kw)


def test_scratch_size_matches_header():
    """The binding's SCRATCH_BYTES is the header's HDC_SCRATCH_BYTES (the no-allocation workspace)."""
    import re
    src = open(os.path.join(ROOT, "include", "hdc.h")).read()
    a, b = re.search(r"#define HDC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src).groups()
    assert hdc.SCRATCH_BYTES == int(a) << int(b)


def test_batch_default_m():
    """The batch's default FFT size (host only): the next power of two (p = 1), except
    4096 (p = 2) for lengths in (4096, 8192]."""
    from paper_2306_10016_amd import tune
    assert [tune.batch_default_m(L) for L in (1, 64, 65, 4096, 4097, 8192, 8193, 65536, 65537)] == \
        [1, 64, 128, 4096, 4096, 4096, 16384, 65536, 131072]


def test_library_binds_torchs_hip_runtime():
    """PyTorch ships its own HIP runtime under the system's soname; loading the library
    first would pull in the system one and leave torch without a device.  The loader
    imports torch first, so a fresh process that touches only the library maps torch's
    runtime (and a single one)."""
    import subprocess
    import sys
    torch = pytest.importorskip("torch")
    import os
    code = ("import sys; sys.path.insert(0, %r); import paper_2306_10016_amd._lib as l; l.lib(); "
            "print('\\n'.join(sorted({x for x in open('/proc/self/maps').read().split() "
            "if x.endswith('libamdhip64.so') or 'libamdhip64.so.' in x})))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    maps = [x for x in out.stdout.split() if x]
    assert len(maps) == 1, maps
    assert os.path.realpath(maps[0]).startswith(os.path.realpath(os.path.dirname(torch.__file__))), maps
