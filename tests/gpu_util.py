"""Helpers shared by the GPU parity tests: seeded inputs, device transfer, tolerances."""
import sys

import numpy as np

import oracle
import synth

TOL = {"c128": 1e-12, "c64": 2e-6}  # relative L2 bars for complex128 / complex64
NP_DT = {"c128": np.complex128, "c64": np.complex64}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(shape, cfg, idx, dtype):
    """Seeded (f, g) in the plan dtype plus their float64 widening for the oracle."""
    f, g = synth.pair(shape, cfg, idx, NP_DT[dtype])
    return f, g, f.astype(np.complex128), g.astype(np.complex128)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def conv1d(plan, f, g):
    ft, gt = to_dev(f), to_dev(g)
    return to_host(plan.convolve(ft, gt))


def rel(a, b):
    return oracle.rel_l2(a, b)
