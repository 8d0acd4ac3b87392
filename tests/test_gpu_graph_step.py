"""Independent convolutions of different sizes (fused and column/row/column plans,
complex and real) captured as one multi-stream HIP graph, as the benchmark replays
its sweep step: every replay, with eager work and synchronisations in between,
must reproduce the eager results bitwise, and those must match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel, say

pytestmark = pytest.mark.gpu

CASES = [  # (L, m, D, dtype)
    (64, 512, 0, "c128"), (1000, 256, 1, "c128"), (3645, 4096, 0, "c128"), (20000, 65536, 0, "c128"),
    (70000, 32768, 2, "c128"), (300000, 1 << 19, 0, "c128"), (5000, 8192, 0, "c64"), (40000, 16384, 0, "r64"),
    (999, 128, 0, "r32"),
]


def test_multistream_graph_replays_match_eager():
    import torch
    import paper_2306_10016_amd as hdc
    dev = torch.device("cuda:0")
    plans, F, G, H, ref = [], [], [], [], []
    for i, (L, m, D, dt) in enumerate(CASES):
        if dt[0] == "r":
            npdt = np.float64 if dt == "r64" else np.float32
            f, g = synth.uniform_real(L, 900, i, 0, npdt), synth.uniform_real(L, 900, i, 1, npdt)
        else:
            f, g = synth.pair(L, 900, i, np.complex128 if dt == "c128" else np.complex64)
        plans.append(hdc.Plan(L, 2 * L - 1, m, 0, 0, 1, D, dt))
        F.append(torch.from_numpy(f).to(dev))
        G.append(torch.from_numpy(g).to(dev))
        H.append(torch.empty(2 * L - 1, dtype=F[-1].dtype, device=dev))
        ref.append(oracle.padded_1d(f.astype(np.complex128), g.astype(np.complex128), 2 * L - 1))
    K = 3
    assign = [list(range(k, len(CASES), K)) for k in range(K)]
    wss = [torch.empty(max([plans[i].workspace_bytes for i in a] + [256]), dtype=torch.uint8, device=dev)
           for a in assign]
    s0 = torch.cuda.Stream()
    streams = [torch.cuda.Stream() for _ in range(K)]

    def body():
        for s in streams:
            s.wait_stream(s0)
        for k, s in enumerate(streams):
            for i in assign[k]:
                plans[i].convolve(F[i], G[i], H[i], ws=wss[k], stream=s)
        for s in streams:
            s0.wait_stream(s)

    with torch.cuda.stream(s0):
        body()
    torch.cuda.synchronize()
    eager = [h.clone() for h in H]
    for i, (L, m, D, dt) in enumerate(CASES):
        err = rel(eager[i].cpu().numpy().astype(np.complex128), ref[i])
        say(f"eager L={L} m={m} {dt}: {err:.2e}")
        assert err < (1e-12 if dt in ("c128", "r64") else 2e-6)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s0, capture_error_mode="thread_local"):
        body()
    for rep in range(4):
        for h in H:
            h.fill_(float("nan"))
        x = torch.ones(1 << 20, device=dev).cumsum(0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        del x
        for i in range(len(CASES)):
            assert torch.equal(H[i], eager[i]), (rep, CASES[i])
        say(f"replay {rep}: all {len(CASES)} outputs equal the eager ones")
