"""Reader for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    L = M = None
    rows = {"f": {}, "g": {}, "h": {}}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("# L="):
                parts = dict(p.split("=") for p in line[2:].split())
                L, M = int(parts["L"]), int(parts["M"])
            if line.startswith("#") or not line.strip():
                continue
            kind, i, re, im = line.split()
            rows[kind][int(i)] = complex(int(re), int(im))
    out = {k: np.array([v[i] for i in range(len(v))], np.complex128) for k, v in rows.items()}
    return L, M, out["f"], out["g"], out["h"]
