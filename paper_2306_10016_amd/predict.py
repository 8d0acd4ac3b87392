"""Learned parameter predictor (section 4.4 and sections 5-6): a small MLP that
maps a problem axis to the scale-free class (p, D) of its best parameters.

* Training data come from the project's own tuner: problems of at most 2^20
  elements (1D with 1, 4 or 16 copies, 2D squares and rectangles, 3D boxes,
  sides of the form 2^a 3^b 5^c 7^d, complex64 and complex128) are tuned one
  axis at a time (the separable search of section 4.2) and every timing is
  cached in the JSON-lines database (section 5.1).
* Classes are scale-free (p, D-mode): p = ceil(L/m) in {1,2,3,4,6,8,12,16},
  D-mode "all residues in one pass" or "one residue per pass".  A class maps
  back to m = the smallest power of two with ceil(L/m) <= p, which is what
  lets a network trained on sides <= 1024 speak about sides of 8192 (the
  "three rays" of m against L in section 6.4.1 are classes of this kind).
* Inference is per axis.  A prediction whose softmax confidence is below a
  threshold falls back to exhaustive per-axis tuning (A0).
* Regret = T(predicted parameters) / T(best of the exhaustive search) - 1.

Run ``python -m paper_2306_10016_amd.predict --out results.json`` on a GPU to
build the database, train the network with the HIP kernels, and evaluate it
on 4096^2, 8192^2 and 256^3 complex64 problems.
"""
from __future__ import annotations

import argparse
import ctypes
import itertools
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import tune

P_CLASSES = tune.P_CLASSES
# dm 0: D = q, 1: D = 1; the last class, p = 0, is explicit padding (q = 1, D = 1)
CLASSES: List[Tuple[int, int]] = [(p, dm) for p in P_CLASSES for dm in (0, 1)] + [(0, 1)]
EXPLICIT = len(CLASSES) - 1
MAX_INNER_M = 1 << 22  # limit of a 1D or innermost axis (column stage 1024 x row stage 4096)
D_IN = 12
SOFT_TAU = 0.03  # soft targets: a class 3 % slower than the best gets weight e^-1
HIDDEN = (128, 128, 128)
MAX_OUTER_M = 1 << 20  # limit of the outer N-D axes (two column stages of at most 1024)


def features(Ls: Sequence[int], axis: int, dtype: str, batch: int = 1) -> np.ndarray:
    """log2 L of this axis, log2 L of the other axes (0 if absent), one-hot axis,
    one-hot ndim, dtype bit, log2 batch (log-sizes scaled by 1/16), and log2 of the
    total element count (scaled by 1/32)."""
    nd = len(Ls)
    others = [Ls[a] for a in range(nd) if a != axis]
    others += [1] * (2 - len(others))
    v = [math.log2(Ls[axis]) / 16.0, math.log2(others[0]) / 16.0, math.log2(others[1]) / 16.0]
    v += [1.0 if axis == a else 0.0 for a in range(3)]
    v += [1.0 if nd == d else 0.0 for d in (1, 2, 3)]
    v += [1.0 if dtype == "c128" else 0.0, math.log2(max(batch, 1)) / 16.0]
    v += [math.log2(max(1, int(np.prod(Ls)) * max(batch, 1))) / 32.0]
    return np.asarray(v, np.float32)


def soft_target(L: int, M: int, table, outer: bool, tau: float = SOFT_TAU) -> np.ndarray:
    """Target distribution over classes from one axis's timing table [((m, D), ms)]:
    weight exp(-(t/t_best - 1)/tau) for every class whose parameters were timed."""
    times = {c: t for c, t in table}
    if not times:
        return np.full(len(CLASSES), 1.0 / len(CLASSES), np.float32)
    tb = min(times.values())
    w = np.zeros(len(CLASSES))
    for ci in range(len(CLASSES)):
        c = params_of(ci, L, M, outer)
        if c in times:
            w[ci] = math.exp(-(times[c] / tb - 1.0) / tau)
    return (w / w.sum()).astype(np.float32)


def class_index(L: int, M: int, m: int, D: int) -> int:
    p = -(-L // m)
    q = -(-M // m)
    if q == 1 and m > 1:
        return EXPLICIT
    # map p to the class whose m is the same power of two
    best = None
    for ci, (pc, dm) in enumerate(CLASSES):
        if tune.m_for_class(L, pc) == m and dm == (0 if D >= q else 1):
            best = ci
            break
    if best is None:
        pc = min(P_CLASSES, key=lambda c: abs(math.log2(c) - math.log2(p)))
        best = CLASSES.index((pc, 0 if D >= q else 1))
    return best


def params_of(ci: int, L: int, M: int, outer: bool) -> Tuple[int, int]:
    """(m, D) for class ci on an axis of length L (outer axes keep m <= 2^20)."""
    pc, dm = CLASSES[ci]
    if ci == EXPLICIT:
        m = tune.pow2_ceil(max(M, 2 * L - 1))
        while m > (MAX_OUTER_M if outer else MAX_INNER_M):
            m //= 2
        while -(-M // m) < -(-L // m):
            m *= 2
        return m, 1
    m = tune.m_for_class(L, pc)
    if outer:
        while m > MAX_OUTER_M:
            m //= 2
    q = -(-M // m)
    p = -(-L // m)
    while q < p:  # keep q >= p
        m *= 2
        q, p = -(-M // m), -(-L // m)
    return m, (q if dm == 0 else 1)


def axis_candidates(L: int, M: int, outer: bool) -> List[Tuple[int, int]]:
    out = []
    for ci in range(len(CLASSES)):
        c = params_of(ci, L, M, outer)
        if c not in out:
            out.append(c)
    return out


# ----------------------------------------------------------- N-D timing --

class NDTimer:
    """Times hdc_convolve of an N-D (or 1D with copies) problem on the GPU."""

    def __init__(self, reps: int = 3, warmup: int = 1):
        self.reps = reps
        self.warmup = warmup
        self._key = None
        self._bufs = None

    def _buffers(self, Ls, Ms, dtype, batch):
        import torch
        from . import torch_dtype, dtype_code
        key = (tuple(Ls), tuple(Ms), dtype, batch)
        if key != self._key:
            self._bufs = None
            td = torch_dtype(dtype_code(dtype))
            n_in = int(np.prod(Ls)) * batch
            n_out = int(np.prod(Ms)) * batch
            self._bufs = (torch.randn(n_in, dtype=td, device="cuda"), torch.randn(n_in, dtype=td, device="cuda"),
                          torch.empty(n_out, dtype=td, device="cuda"))
            self._key = key
        return self._bufs

    def __call__(self, Ls, Ms, ms, Ds, dtype, batch=1) -> float:
        from . import Plan
        f, g, h = self._buffers(Ls, Ms, dtype, batch)
        if len(Ls) == 1:
            plan = Plan(Ls[0], Ms[0], ms[0], 0, 0, batch, Ds[0], dtype)
        else:
            plan = Plan.nd(Ls, Ms, ms, D=Ds, dtype=dtype)
        ws = tune._shared_ws(plan.workspace_bytes)
        t = plan.time_convolve(f, g, h, ws=ws, warmup=self.warmup, reps=self.reps)
        plan.close()
        t.sort()
        return t[len(t) // 2]


def default_params(Ls, Ms):
    """The method without the predictor: p = 1 (m = next power of two >= L), all residues at once."""
    out = []
    for a, (L, M) in enumerate(zip(Ls, Ms)):
        out.append(params_of(CLASSES.index((1, 0)), L, M, outer=a < len(Ls) - 1))
    return out


def tune_separable(Ls, Ms, dtype, timer, batch=1, db: Optional[tune.TuneDB] = None):
    """A0 per axis (section 4.2): each axis searched with the others at their defaults.
    Returns (per-axis best (m, D), per-axis tables, time of the combined choice)."""
    from . import HdcError
    base = default_params(Ls, Ms)
    best, tables = [], []
    for a in range(len(Ls)):
        rows = []
        for c in axis_candidates(Ls[a], Ms[a], outer=a < len(Ls) - 1):
            cur = list(base)
            cur[a] = c
            try:
                t = timer(Ls, Ms, [x[0] for x in cur], [x[1] for x in cur], dtype, batch)
            except HdcError as e:  # a parameter set the kernels do not implement
                print(f"[tune] skip {Ls} axis {a} {c}: {e}", flush=True)
                continue
            rows.append((c, t))
            if db is not None:
                db.add(tune.problem_key(list(Ls), list(Ms), dtype, batch),
                       {"axis": a, "m": [x[0] for x in cur], "D": [x[1] for x in cur]}, t)
        rows.sort(key=lambda r: (r[1], r[0][0], r[0][1]))
        best.append(rows[0][0] if rows else base[a])
        tables.append(rows)
    t = timer(Ls, Ms, [b[0] for b in best], [b[1] for b in best], dtype, batch)
    return best, tables, t


def tune_joint(Ls, Ms, dtype, timer, batch=1):
    """Exhaustive search over the product of the per-axis candidate sets (the reference point of the regret).
    For 3D problems the product is limited to the all-residues mode (D = q) on every
    axis, which keeps it at (#m)^3 combinations."""
    from . import HdcError
    cands = [axis_candidates(L, M, outer=a < len(Ls) - 1) for a, (L, M) in enumerate(zip(Ls, Ms))]
    if len(Ls) == 3:
        cands = [[c for c in cs if c[1] == -(-M // c[0])] for cs, M in zip(cands, Ms)]
    rows = []
    for combo in itertools.product(*cands):
        try:
            t = timer(Ls, Ms, [c[0] for c in combo], [c[1] for c in combo], dtype, batch)
        except HdcError:
            continue
        rows.append((list(combo), t))
    rows.sort(key=lambda r: r[1])
    return rows


# ------------------------------------------------------------ predictor --

class Predictor:
    def __init__(self, seed: int = 0, threshold: float = 0.0):
        from .mlp import MLP
        self.net = MLP([D_IN, *HIDDEN, len(CLASSES)], seed=seed)
        self.threshold = threshold
        self.history: List[float] = []
        self.lo = self.hi = None  # training range of the features (set by fit)

    def fit(self, X: np.ndarray, y: np.ndarray, epochs: int = 300, lr: float = 2e-3, batch: int = 128):
        """Train on labels y (n,) or on target distributions y (n x K); remembers the
        training range of every feature."""
        soft = y.ndim == 2
        self.lo, self.hi = X.min(axis=0).astype(np.float32), X.max(axis=0).astype(np.float32)
        self.history = self.net.train(X, y, epochs=epochs, batch=batch, lr=lr, soft=soft)
        return self.history

    def save(self, path: str) -> None:
        """Checkpoint for hdc_predictor_load (see save_checkpoint), with the training
        range when the network has been fitted."""
        save_checkpoint(path, self.net.host_params(), self.lo, self.hi)

    def predict_axes(self, Ls, Ms, dtype, batch=1):
        """Per-axis (m, D), the per-axis confidence, and the class indices."""
        X = np.stack([features(Ls, a, dtype, batch) for a in range(len(Ls))])
        P = self.net.predict_proba(X)
        out, conf, cls = [], [], []
        for a in range(len(Ls)):
            ci = int(np.argmax(P[a]))  # ties: lowest class index
            out.append(params_of(ci, Ls[a], Ms[a], outer=a < len(Ls) - 1))
            # an axis outside the training range abstains (confidence 0)
            conf.append(float(P[a, ci]) if in_range(X[a], self.lo, self.hi) else 0.0)
            cls.append(ci)
        return out, conf, cls

    def shortlist(self, Ls, Ms, dtype, k=2, batch=1):
        """Per axis, the parameters of the k most probable distinct classes."""
        X = np.stack([features(Ls, a, dtype, batch) for a in range(len(Ls))])
        P = self.net.predict_proba(X)
        out = []
        for a in range(len(Ls)):
            cands = []
            for ci in np.argsort(-P[a], kind="stable"):
                c = params_of(int(ci), Ls[a], Ms[a], outer=a < len(Ls) - 1)
                if c not in cands:
                    cands.append(c)
                if len(cands) == k:
                    break
            out.append(cands)
        return out

    def choose(self, Ls, Ms, dtype, timer, batch=1):
        """Predicted parameters, or exhaustive per-axis tuning when confidence is low
        (an axis outside the training range has confidence 0)."""
        params, conf, _ = self.predict_axes(Ls, Ms, dtype, batch)
        if min(conf) < max(self.threshold, 1e-6):
            best, _, _ = tune_separable(Ls, Ms, dtype, timer, batch)
            return best, "fallback"
        return params, "predicted"


FEATURE_VERSION = 1
# features outside the training range by more than this (in the scaled units of
# features(): 1/16 of an octave for lengths) make the network abstain on that axis
RANGE_MARGIN = 1.0 / 16


def save_checkpoint(path: str, params, lo=None, hi=None) -> None:
    """Write a network [(W, b), ...] (W out x in) in the checkpoint format that
    hdc_predictor_load reads (include/hdc_tune.h): "HDCMLP01", int32 format
    version (1, or 2 with the training range), int32 layer count n, int32
    sizes[n + 1], then W and b of every layer as float32, and for version 2 the
    per-feature minimum and maximum over the training rows (float32), little
    endian."""
    import struct
    sizes = [int(params[0][0].shape[1])] + [int(W.shape[0]) for W, _ in params]
    ver = 1 if lo is None else 2
    with open(path, "wb") as fh:
        fh.write(b"HDCMLP01")
        fh.write(struct.pack("<ii", ver, len(params)))
        fh.write(struct.pack("<%di" % len(sizes), *sizes))
        for W, b in params:
            fh.write(np.ascontiguousarray(W, dtype="<f4").tobytes())
            fh.write(np.ascontiguousarray(b, dtype="<f4").tobytes())
        if ver == 2:
            fh.write(np.ascontiguousarray(lo, dtype="<f4").tobytes())
            fh.write(np.ascontiguousarray(hi, dtype="<f4").tobytes())


def in_range(x: np.ndarray, lo: Optional[np.ndarray], hi: Optional[np.ndarray]) -> bool:
    """Whether a feature row lies inside the training range (within RANGE_MARGIN)."""
    if lo is None:
        return True
    return bool(np.all(x >= lo - RANGE_MARGIN) and np.all(x <= hi + RANGE_MARGIN))


class CheckpointPredictor:
    """A saved network evaluated by the library (hdc_predictor_load / hdc_predict):
    per-axis features, the MLP forward in the HIP kernels, and the class-to-
    parameter mapping all run behind the C boundary."""

    def __init__(self, path: str):
        from ._lib import lib, check
        self._lib = lib()
        h = ctypes.c_void_p()
        check(self._lib.hdc_predictor_load(ctypes.byref(h), path.encode()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdc_predictor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def predict_axes(self, Ls, Ms, dtype, batch=1):
        """Per-axis (m, D) and confidence from hdc_predict."""
        from ._lib import Params, check
        pr = tune.problem(list(Ls), list(Ms), dtype, batch)
        out = Params()
        conf = (ctypes.c_float * 3)()
        check(self._lib.hdc_predict(self._h, ctypes.byref(pr), ctypes.byref(out), conf))
        nd = len(Ls)
        return [(int(out.m[a]), int(out.D[a])) for a in range(nd)], [float(conf[a]) for a in range(nd)]


def smooth_sides(lo: int, hi: int) -> List[int]:
    out = []
    for a in range(0, 21):
        for b in range(0, 13):
            for c in range(0, 9):
                for d in range(0, 8):
                    v = 2 ** a * 3 ** b * 5 ** c * 7 ** d
                    if lo <= v <= hi:
                        out.append(v)
    return sorted(set(out))


def training_problems(seed: int = 0, max_elems: int = 1 << 20):
    """(Ls, batch, dtype) training problems of at most max_elems elements."""
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([230610016, 5, seed])))
    probs = []
    s1 = smooth_sides(64, max_elems)
    for dt in ("c64", "c128"):
        for L in r.choice(s1, size=min(40, len(s1)), replace=False):
            for batch in (1, 4, 16):
                if L * batch <= max_elems:
                    probs.append(([int(L)], batch, dt))
        s2 = smooth_sides(16, 1024)
        for _ in range(36):
            x, y = int(r.choice(s2)), int(r.choice(s2))
            if x * y <= max_elems:
                probs.append(([x, y], 1, dt))
        for L in (128, 256, 512, 1024):  # squares and L_y = 32 rectangles (section 6.4)
            probs.append(([L, L], 1, dt))
            probs.append(([L, 32], 1, dt))
        # skinny rectangles and bars with one long axis (section 5.1's rectangles,
        # section 6.4's L_y = 32 heuristic): full-length axes within 2^20 elements
        s_long = smooth_sides(1024, 16384)
        for L in r.choice(s_long, size=min(10, len(s_long)), replace=False).tolist() + [4096, 8192, 16384]:
            for w in (16, 32):
                if L * w <= max_elems:
                    probs.append(([int(L), w], 1, dt))
                    probs.append(([w, int(L)], 1, dt))
        for L in (256, 512, 1024, 2048, 4096):
            for pos in range(3):
                dims = [16, 16, 16]
                dims[pos] = L
                probs.append((dims, 1, dt))
        # outer axes of moderate length over many copies (the inner axis long), and
        # boxes whose every axis runs over a few thousand copies
        for Lo in (64, 128, 256, 512):
            for Li in (2048, 4096, 8192, 16384):
                if Lo * Li <= max_elems:
                    probs.append(([Lo, Li], 1, dt))
        for dims in ([32, 32, 1024], [64, 64, 256], [32, 128, 256], [128, 64, 128], [64, 128, 128]):
            probs.append((list(dims), 1, dt))
        s3 = smooth_sides(8, 101)
        for _ in range(12):
            dims = [int(r.choice(s3)) for _ in range(3)]
            if int(np.prod(dims)) <= max_elems:
                probs.append((dims, 1, dt))
    # large 2D and 3D problems (2^22 .. 2^26 elements, section 5.1's smooth sides):
    # where the copies of an outer axis fill the GPU by themselves
    for dims in LARGE_PROBLEMS:
        probs.append((list(dims), 1, "c64"))
    for dims in LARGE_PROBLEMS[::3]:
        probs.append((list(dims), 1, "c128"))
    return probs


# large training problems: none is an evaluation problem
LARGE_PROBLEMS = [(2048, 2048), (3000, 3000), (3375, 3375), (5000, 5000), (6144, 6144), (7000, 7000),
                  (2048, 8192), (8192, 2048), (4096, 8192), (8192, 4096), (6000, 4000), (1024, 16384),
                  (16384, 1024), (4096, 2048), (2048, 4096), (12000, 2500), (2500, 12000), (3000, 6000),
                  (128, 128, 128), (192, 192, 192), (200, 200, 200), (300, 300, 300), (320, 320, 320),
                  (128, 256, 256), (256, 128, 256), (256, 256, 128), (384, 256, 256), (256, 256, 384),
                  (512, 256, 128), (128, 512, 512)]


EVAL_PROBLEMS = [([4096, 4096], "c64"), ([8192, 8192], "c64"), ([256, 256, 256], "c64")]
# problems inside the training range that training never saw (1D lengths just above a
# power of two, where p = 1 pads to almost four times L, and 2D rectangles)
HELDOUT_PROBLEMS = [([4100], "c128"), ([8300], "c128"), ([17000], "c128"), ([33000], "c64"), ([66000], "c64"),
                    ([131100], "c128"), ([600, 130], "c64"), ([96, 3000], "c128"), ([1100, 700], "c64")]
DEFAULT_CKPT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "predictor.bin")


def time_params(Ls, Ms, dtype, params, reps: int = 5, warmup: int = 2, _bufs={}) -> float:
    """Median time of one parameter set {"m", "D", "tile"} (hdc_plan_params + hdc_time_convolve)."""
    import torch
    from . import Plan, torch_dtype, dtype_code
    key = (tuple(Ls), tuple(Ms), dtype)
    if key not in _bufs:
        _bufs.clear()
        td = torch_dtype(dtype_code(dtype))
        _bufs[key] = (torch.randn(int(np.prod(Ls)), dtype=td, device="cuda"),
                      torch.randn(int(np.prod(Ls)), dtype=td, device="cuda"),
                      torch.empty(int(np.prod(Ms)), dtype=td, device="cuda"))
    f, g, h = _bufs[key]
    L_arg = list(Ls) if len(Ls) > 1 else Ls[0]
    M_arg = list(Ms) if len(Ms) > 1 else Ms[0]
    plan = Plan.from_params(L_arg, M_arg, dtype, params)
    t = plan.time_convolve(f, g, h, ws=tune._shared_ws(plan.workspace_bytes), warmup=warmup, reps=reps)
    plan.close()
    t.sort()
    return t[len(t) // 2]


def as_params(pairs, nd):
    """[(m, D), ...] per axis -> {"m", "D"} in the database's form (scalars for 1D)."""
    if nd == 1:
        return {"m": int(pairs[0][0]), "D": int(pairs[0][1])}
    return {"m": [int(p[0]) for p in pairs], "D": [int(p[1]) for p in pairs]}


def evaluate(pred, problems, log=print):
    """Per problem: the library's exhaustive search (A0, section 4.2) as the judge, the
    network's top-1 parameters (abstaining axes marked), the flow with the A0 fallback,
    and the default (p = 1, all residues) -- all re-timed under the same conditions."""
    out = []
    for Ls, dt in problems:
        Ms = [2 * L - 1 for L in Ls]
        a0, _ = tune.run_search(tune.TuneDB(None), Ls if len(Ls) > 1 else Ls[0],
                                Ms if len(Ms) > 1 else Ms[0], dt, tune.A0)
        t_a0 = time_params(Ls, Ms, dt, a0.params)
        params, conf = pred.predict_axes(Ls, Ms, dt)[:2]
        t_net = time_params(Ls, Ms, dt, as_params(params, len(Ls)))
        abstain = min(conf) <= 0.0
        dflt = default_params(Ls, Ms)
        t_def = time_params(Ls, Ms, dt, as_params(dflt, len(Ls)))
        ent = {"L": Ls, "dtype": dt, "A0": {"params": a0.params, "ms": t_a0, "timings": len(a0.table)},
               "network": {"params": params, "confidence": conf, "ms": t_net, "regret": tune.regret(t_net, t_a0)},
               "abstained": abstain,
               "flow": {"source": "A0 fallback" if abstain else "network",
                        "regret": 0.0 if abstain else tune.regret(t_net, t_a0)},
               "default": {"params": dflt, "ms": t_def, "regret": tune.regret(t_def, t_a0)}}
        out.append(ent)
        log(f"[predict] {Ls} {dt}: A0 {t_a0:.4f} ms ({len(a0.table)} timings); network {params} "
            f"{'abstains' if abstain else 'conf %.2f' % min(conf)}, regret {ent['network']['regret']:+.3f}; "
            f"default regret {ent['default']['regret']:+.3f}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", default="results/predictor_db.jsonl")
    ap.add_argument("--out", default="results/predictor.json")
    ap.add_argument("--ckpt", default=DEFAULT_CKPT)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--max-problems", type=int, default=0)
    args = ap.parse_args(argv)
    timer = NDTimer(reps=3, warmup=1)
    db = tune.TuneDB(args.db, device=tune.device_name(), build=tune.build_hash())
    probs = training_problems()
    if args.max_problems:
        probs = probs[:args.max_problems]
    X, y, T, meta = [], [], [], []
    t0 = time.time()
    for i, (Ls, batch, dt) in enumerate(probs):
        Ms = [2 * L - 1 for L in Ls]
        best, tables, _ = tune_separable(Ls, Ms, dt, timer, batch, db)
        for a in range(len(Ls)):
            X.append(features(Ls, a, dt, batch))
            y.append(class_index(Ls[a], Ms[a], best[a][0], best[a][1]))
            T.append(soft_target(Ls[a], Ms[a], tables[a], outer=a < len(Ls) - 1))
        meta.append({"L": Ls, "batch": batch, "dtype": dt, "best": best})
        if i % 25 == 0:
            print(f"[predict] tuned {i + 1}/{len(probs)} ({time.time() - t0:.0f} s)", flush=True)
    X = np.stack(X)
    y = np.asarray(y, np.int32)
    T = np.stack(T)
    pred = Predictor(seed=0)
    hist = pred.fit(X, T, epochs=args.epochs)  # soft targets from the timing tables
    train_acc = float(np.mean(np.argmax(pred.net.predict_proba(X), 1) == y))
    print(f"[predict] trained: loss {hist[0]:.3f} -> {hist[-1]:.3f}, train accuracy {train_acc:.3f}", flush=True)
    os.makedirs(os.path.dirname(args.ckpt) or ".", exist_ok=True)
    pred.save(args.ckpt)
    results = {"train": {"problems": len(probs), "rows": int(len(y)), "loss_first": hist[0], "loss_last": hist[-1],
                         "accuracy": train_acc, "class_counts": np.bincount(y, minlength=len(CLASSES)).tolist(),
                         "seconds": round(time.time() - t0, 1)},
               "checkpoint": os.path.relpath(args.ckpt, os.path.dirname(os.path.dirname(os.path.abspath(__file__)))),
               "eval": evaluate(pred, EVAL_PROBLEMS), "heldout": evaluate(pred, HELDOUT_PROBLEMS)}
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    json.dump(results, open(args.out, "w"), indent=1)
    for part in ("eval", "heldout"):
        e = results[part]
        print(json.dumps({part: [{"L": x["L"], "network": round(x["network"]["regret"], 4), "abstained": x["abstained"],
                                  "default": round(x["default"]["regret"], 4)} for x in e]}), flush=True)


if __name__ == "__main__":
    main()
