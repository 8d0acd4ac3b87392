"""The parameter studies of sections 5.2 and 6.4, rerun on this build's own GPU timings.

Both ask how well a cheap rectangle L_x x L_y predicts the best x-axis FFT size m
of the square L_x x L_x (the x axis is the outer, column-pass axis of the 2D plan;
every candidate runs all residues at once and the y axis keeps its default).

* epsilon threshold (section 5.2).  The square's timings t_s(m) give its best
  m*_s, t*_s and worst t^w_s.  The threshold is read as
      gamma(eps) = t*_s + eps (t^w_s - t*_s)
  (the printed formula is garbled: it subtracts the worst time from the best,
  which would put the threshold below the best time).  A rectangle predicts the
  square at eps when the m it finds fastest for itself, run on the square, is
  within gamma(eps); the study reports the smallest such L_y over smooth heights
  (2^a 3^b 5^c 7^d) for each square and eps.
* fixed height (section 6.4).  The rectangle of height h (4, 8, 16, 32) chooses
  m; its regret on the square is t_s(m*_r) / t*_s - 1.

    python -m paper_2306_10016_amd.study --out profiles/epsilon_study.json
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

EPSILONS = (0.00005, 0.001, 0.01, 0.05, 0.1)
HEIGHTS = (4, 8, 16, 32)


def gamma(ts: Dict[int, float], eps: float) -> float:
    """The time threshold of the square at eps: t* + eps (t_worst - t*)."""
    best, worst = min(ts.values()), max(ts.values())
    return best + eps * (worst - best)


def choice(tr: Dict[int, float]) -> int:
    """The rectangle's choice: its fastest m (ties: the smaller m)."""
    return min(tr, key=lambda m: (tr[m], m))


def smallest_predicting_height(ts: Dict[int, float], rects: Sequence[Tuple[int, Dict[int, float]]],
                               eps: float) -> Optional[int]:
    """The smallest height L_y among `rects` ((L_y, timings) pairs) whose choice runs on
    the square within gamma(eps); None if no rectangle does."""
    g = gamma(ts, eps)
    for Ly, tr in sorted(rects, key=lambda r: r[0]):
        m = choice(tr)
        if m in ts and ts[m] <= g:
            return Ly
    return None


def height_regret(ts: Dict[int, float], tr: Dict[int, float]) -> float:
    """Regret on the square of the rectangle's choice: t_s(m*_r) / t*_s - 1."""
    return ts[choice(tr)] / min(ts.values()) - 1.0


def run(squares: Sequence[int], max_height: int = 256, dtype: str = "c64", reps: int = 3) -> dict:
    """Time the x-axis candidates on every square and rectangle and evaluate both studies."""
    from . import HdcError
    from .predict import NDTimer, axis_candidates, default_params, smooth_sides
    timer = NDTimer(reps=reps, warmup=1)

    def table(Lx: int, Ly: int) -> Dict[int, float]:
        Ls, Ms = [Lx, Ly], [2 * Lx - 1, 2 * Ly - 1]
        ydef = default_params(Ls, Ms)[1]
        out = {}
        for m, D in axis_candidates(Lx, Ms[0], outer=True):
            if D != -(-Ms[0] // m):  # all residues at once
                continue
            try:
                out[m] = timer(Ls, Ms, [m, ydef[0]], [D, ydef[1]], dtype)
            except HdcError:
                continue
        return out

    res = {"dtype": dtype, "epsilons": list(EPSILONS), "heights": list(HEIGHTS), "squares": []}
    for Lx in squares:
        ts = table(Lx, Lx)
        heights = sorted(set(smooth_sides(2, min(Lx, max_height))) | set(h for h in HEIGHTS if h <= Lx))
        rects = [(Ly, table(Lx, Ly)) for Ly in heights]
        ent = {"Lx": Lx, "square": {str(m): t for m, t in ts.items()}, "m_best": choice(ts),
               "rect_choice": {str(Ly): choice(tr) for Ly, tr in rects},
               "smallest_Ly": {str(e): smallest_predicting_height(ts, rects, e) for e in EPSILONS},
               "fixed_height_regret": {str(h): height_regret(ts, tr) for h, tr in rects if h in HEIGHTS}}
        res["squares"].append(ent)
        print(f"[study] Lx={Lx}: best m {ent['m_best']}, smallest Ly {ent['smallest_Ly']}, "
              f"fixed-height regret {ent['fixed_height_regret']}", flush=True)
    return res


def main(argv: Optional[List[str]] = None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join("results", "epsilon_study.json"))
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--squares", default="243,256,343,512,625,1024,1125,2048")
    ap.add_argument("--max-height", type=int, default=256)
    args = ap.parse_args(argv)
    res = run([int(x) for x in args.squares.split(",")], args.max_height, args.dtype)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    json.dump(res, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
