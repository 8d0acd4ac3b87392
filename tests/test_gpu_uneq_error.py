"""Accuracy of the unequal-length convolution as the longer operand grows, for a
fixed shorter operand of length 2 or 12 and several transform lengths: the
study of the L2 error against the length of g (section 6.1's figure on padding
sizes).  The reference is the oracle's FP64 direct sum; explicit padding
(torch.fft on the GPU, the same dtype) is measured beside it.  The bar is the
normwise bound of FFT-based convolution, a small multiple of eps log2 N."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import NP_DT, rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

EPS = {"c128": 2.0 ** -53, "c64": 2.0 ** -24}
LG = [64, 243, 1024, 3125, 16384, 59049, 262144, 823543, 1 << 22]


def _explicit(ft, gt, M):
    import torch
    n = 1 << (M - 1).bit_length()
    return torch.fft.ifft(torch.fft.fft(ft, n) * torch.fft.fft(gt, n))[:M]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("Lf", [2, 12])
def test_error_vs_length(Lf, dtype):
    import paper_2306_10016_amd as hdc
    rows = []
    for i, Lg in enumerate(LG):
        M = Lf + Lg - 1
        f = synth.uniform_complex(Lf, 700, i, 0, NP_DT[dtype])
        g = synth.uniform_complex(Lg, 700, i, 1, NP_DT[dtype])
        ref = oracle.direct_1d(f.astype(np.complex128), g.astype(np.complex128), M)
        ft, gt = to_dev(f), to_dev(g)
        s, l, _ = hdc.uneq_derive(Lf, Lg, M)
        # transform lengths: the derived default, the fewest residues (Lambda m = 2^ceil(log2 M)
        # up to 2^22) and four times as many
        variants = {"default": (0, 0)}
        mg1 = min(1 << (M - 1).bit_length(), 1 << 22)
        variants["q1"] = (max(1, mg1 // min(1024, max(1, mg1 // 64))), min(1024, max(1, mg1 // 64)))
        mg4 = max(1, mg1 // 4)
        if 4 * mg4 >= Lg:
            variants["q4"] = (max(1, mg4 // min(1024, max(1, mg4 // 64))), min(1024, max(1, mg4 // 64)))
        row = {"Lg": Lg}
        for name, (m, lam) in variants.items():
            plan = hdc.UneqPlan(Lf, Lg, M, m=m, lam=lam, dtype=dtype)
            N = plan.axes[0]["N"]
            e = rel(to_host(plan.convolve(ft, gt)), ref)
            bound = 4 * EPS[dtype] * math.log2(N) + 8 * EPS[dtype]
            assert e < bound, (name, Lg, e, bound)
            row[name] = (N, e)
        row["explicit"] = rel(to_host(_explicit(ft, gt, M)), ref)
        rows.append(row)
    say(f"\nL2 error vs Lg, Lf = {Lf}, {dtype} (N: relative error)")
    for r in rows:
        parts = "  ".join(f"{k} N={v[0]}: {v[1]:.2e}" for k, v in r.items() if isinstance(v, tuple))
        say(f"  Lg={r['Lg']:>8}  {parts}  explicit: {r['explicit']:.2e}")
