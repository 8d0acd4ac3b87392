"""Writes the stored expected values under tests/golden/.

Calls only the oracle (and the seeded input generator).  Inputs are Gaussian
integers, so the direct sum of eq. (5) is exact in FP64 and the stored
outputs are exact integers.

fig2_L6_M11.txt -- the worked shape of the paper's 1D parameter figure
(section 2.5, Fig. 2): L = 6, M = 11, m = 4, so p = 2 and q = 3.  The paper
prints the shape only, no values.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def write_case(name, L, M, cfg, size_idx, bound, note):
    f = synth.gaussian_integers(L, bound, cfg, size_idx, 0)
    g = synth.gaussian_integers(L, bound, cfg, size_idx, 1)
    h = oracle.direct_1d(f, g, M)
    with open(os.path.join(HERE, name), "w") as fh:
        fh.write(f"# {note}\n# L={L} M={M}\n# columns: kind index re im\n")
        for kind, arr in (("f", f), ("g", g), ("h", h)):
            for i, z in enumerate(arr):
                fh.write(f"{kind} {i} {int(z.real)} {int(z.imag)}\n")


if __name__ == "__main__":
    write_case("fig2_L6_M11.txt", 6, 11, 120, 0, 8,
               "section 2.5, Fig. 2 shape (L=6, M=11, m=4, p=2, q=3); Gaussian-integer inputs, exact output")
    write_case("int_L37_M80.txt", 37, 80, 120, 1, 8,
               "ragged shape L=37, M=80 (M > 2L-1: zero tail); Gaussian-integer inputs, exact output")
