"""Experience-based autotuner for the hybrid-dealiasing parameters (section 4).

The searches run in the library (hdc_tune / hdc_tune_host of
include/hdc_tune.h); this module marshals arguments and reads the timing
database back:

* **A0** (section 4.2): exhaustive grid over the candidate FFT sizes m (each
  fixing p = ceil(L/m), q = ceil(M/m)), residues per pass D and, for the best,
  the column tile.  N-D problems are searched one axis at a time with the
  other axes at their defaults (the per-dimension separability of section 4.2).
* **A1** (section 4.3, "experience"): (1) reuse the best entry of the timing
  database for the same problem; (2) seed with the scale-free classes (p, D)
  that won on the nearest already-tuned problems; (3) random candidates; (4)
  local refinement around the best so far (the neighbouring m and D).

Every candidate is scored by the measured time of the whole convolution (HIP
events, median of 5 after 2 warm-ups), or by a caller's cost function
(``timer=``, host only: the searches' CPU tests).  All timings are appended to
a JSON-lines database (section 5.1 keeps every measured result), keyed by
problem, parameters, device and library build, so a killed run resumes where
it stopped.  The unequal-length tuner and the per-bucket batch tuner below
remain Python searches over the timing entry point.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import random
import tempfile
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

P_CLASSES = (1, 2, 3, 4, 6, 8, 12, 16)
A0, A1 = 0, 1


def pow2_ceil(x: int) -> int:
    m = 1
    while m < x:
        m <<= 1
    return m


def scale_class(L: int, M: int, m: int, D: int) -> Tuple[int, int]:
    """Scale-free class of a parameter set: (p, D relative to q) -- section 6.4's rays."""
    p = -(-L // m)
    q = -(-M // m)
    return (p, 0 if D >= q else D)


def m_for_class(L: int, p: int) -> int:
    """Smallest power-of-two m with ceil(L/m) <= p."""
    return pow2_ceil(-(-L // p))


def build_hash() -> str:
    """This library build's identity (hdc_build_id), as the tuner records it in the database."""
    from ._lib import lib
    return lib().hdc_build_id().decode()


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def problem_key(L, M, dtype: str, batch: int = 1) -> str:
    Ls = list(L) if isinstance(L, (list, tuple)) else [int(L)]
    Ms = list(M) if isinstance(M, (list, tuple)) else [int(M)]
    return json.dumps({"L": Ls, "M": Ms, "dtype": dtype, "batch": int(batch)}, sort_keys=True)


class TuneDB:
    """Append-only JSON-lines timing database shared with the library's tuner.

    ``path=None`` keeps the database in a temporary file for the life of this
    object (the library reads and appends it on every search).  ``device`` /
    ``build`` select the rows that count ("any" accepts every value)."""

    def __init__(self, path: Optional[str] = None, device: Optional[str] = None, build: Optional[str] = None):
        self._tmp = None
        if path is None:
            fd, path = tempfile.mkstemp(prefix="hdc_tune_", suffix=".jsonl")
            os.close(fd)
            self._tmp = path
        self.path = path
        self.device = device or "any"
        self.build = build or "any"
        self.rows: List[dict] = []
        self.reload()

    def __del__(self):
        if getattr(self, "_tmp", None):
            try:
                os.unlink(self._tmp)
            except OSError:
                pass

    def reload(self):
        self.rows = []
        if os.path.exists(self.path):
            with open(self.path) as fh:
                for line in fh:
                    line = line.strip()
                    if not line:
                        continue
                    try:
                        r = json.loads(line)
                    except (ValueError, RecursionError):  # JSONDecodeError is a ValueError
                        continue  # a line cut short by a kill, or not a row
                    # rows of this form only (a hand-edited or foreign line is skipped)
                    if isinstance(r, dict) and isinstance(r.get("key"), str) and isinstance(r.get("params"), dict) \
                            and isinstance(r.get("ms"), (int, float)) and not isinstance(r.get("ms"), bool):
                        self.rows.append(r)

    def add(self, key: str, params: dict, ms: float, extra: Optional[dict] = None):
        row = {"key": key, "params": params, "ms": float(ms), "device": self.device, "build": self.build,
               "t": time.time()}
        if extra:
            row.update(extra)
        self.rows.append(row)
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(self.path, "a") as fh:
            fh.write(json.dumps(row) + "\n")

    def _mine(self, r):
        return (self.device == "any" or r.get("device") == self.device) and \
            (self.build == "any" or r.get("build") == self.build)

    def timings(self, key: str) -> Dict[str, float]:
        out = {}
        for r in self.rows:
            if r["key"] == key and self._mine(r):
                pk = json.dumps(r["params"], sort_keys=True)
                out[pk] = min(out.get(pk, math.inf), r["ms"])
        return out

    def best(self, key: str) -> Optional[Tuple[dict, float]]:
        t = self.timings(key)
        if not t:
            return None
        pk = min(t, key=lambda k: (t[k], k))
        return json.loads(pk), t[pk]

    def keys(self):
        return sorted({r["key"] for r in self.rows if self._mine(r)})


@dataclass
class TuneResult:
    params: dict
    ms: float
    table: List[Tuple[dict, float]] = field(default_factory=list)
    source: str = "search"


def problem(L, M, dtype: str, batch: int = 1):
    """hdc_problem of a 1D (int L) or N-D (sequence L) problem."""
    from . import dtype_code
    from ._lib import Problem
    Ls = list(L) if isinstance(L, (list, tuple)) else [int(L)]
    Ms = list(M) if isinstance(M, (list, tuple)) else [int(M)]
    pr = Problem()
    pr.ndim = len(Ls)
    for a in range(len(Ls)):
        pr.L[a], pr.M[a] = int(Ls[a]), int(Ms[a])
    pr.dtype = dtype_code(dtype)
    pr.batch = int(batch)
    return pr


def params_dict(prm, ndim: int) -> dict:
    """hdc_params as the database writes it: {"m", "D"} (+ "tile" when not the default),
    scalars for 1D and per-axis lists for N-D."""
    if ndim == 1:
        d = {"m": int(prm.m[0]), "D": int(prm.D[0])}
        if prm.tile[0]:
            d["tile"] = int(prm.tile[0])
        return d
    d = {"m": [int(prm.m[a]) for a in range(ndim)], "D": [int(prm.D[a]) for a in range(ndim)]}
    if any(prm.tile[a] for a in range(ndim)):
        d["tile"] = [int(prm.tile[a]) for a in range(ndim)]
    return d


def run_search(db: TuneDB, L, M, dtype: str, mode: int, timer: Optional[Callable] = None, batch: int = 1):
    """One search of the library's tuner (mode A0 or A1) on problem (L, M, dtype, batch).
    ``timer(prob, params) -> ms`` (ctypes records) replaces the GPU timing: hdc_tune_host.
    Returns (TuneResult, the hdc_params chosen)."""
    from ._lib import COST_FN, Params, check, lib
    pr = problem(L, M, dtype, batch)
    key = problem_key(L, M, dtype, batch)
    db.reload()
    before = len(db.timings(key))
    best, ms = Params(), ctypes.c_double()
    if timer is None:
        check(lib().hdc_tune(ctypes.byref(pr), mode, db.path.encode(), ctypes.byref(best), ctypes.byref(ms)))
    else:
        def cost(pp, pm, _ctx):
            try:
                return float(timer(pp.contents, pm.contents))
            except Exception:  # an exception cannot cross the C boundary: report the set as unusable
                return -1.0
        cb = COST_FN(cost)
        check(lib().hdc_tune_host(ctypes.byref(pr), mode, db.path.encode(), db.device.encode(), db.build.encode(),
                                  cb, None, ctypes.byref(best), ctypes.byref(ms)))
    db.reload()
    table = [(json.loads(pk), t) for pk, t in db.timings(key).items()]
    source = ("db" if (mode == A1 and before > 0 and len(table) == before) else ("A0" if mode == A0 else "A1"))
    return TuneResult(params_dict(best, pr.ndim), float(ms.value), table, source), best


class Tuner1D:
    """Tunes a 1D problem (L, M, dtype) with the library's searches.

    ``timer(L, M, m, D, dtype) -> ms`` replaces the GPU timing (host-only
    searches through hdc_tune_host); by default every candidate is timed on the
    GPU by hdc_tune."""

    def __init__(self, db: Optional[TuneDB] = None, reps: int = 5, warmup: int = 2,
                 timer: Optional[Callable[[int, int, int, int, str], float]] = None):
        self.db = db or TuneDB(None)
        self.reps = reps      # for measure(): the searches time with 2 warm-ups and 5 runs
        self.warmup = warmup
        self.timer = timer
        self._bufs = {}

    def _search(self, mode, L, M, dtype, batch=1):
        t = None
        if self.timer is not None:
            def t(pr, pm):
                return self.timer(int(pr.L[0]), int(pr.M[0]), int(pm.m[0]), int(pm.D[0]), dtype)
        return run_search(self.db, L, M, dtype, mode, t, batch)[0]

    def a0(self, L: int, M: int, dtype: str = "c128", batch: int = 1) -> TuneResult:
        """Exhaustive search (section 4.2)."""
        return self._search(A0, L, M, dtype, batch)

    def a1(self, L: int, M: int, dtype: str = "c128", batch: int = 1) -> TuneResult:
        """Experience search (section 4.3)."""
        return self._search(A1, L, M, dtype, batch)

    def measure(self, L, M, m, D, dtype, tile: int = 0) -> float:
        """Median time of one parameter set (the caller's timer, or hdc_time_convolve)."""
        if self.timer is not None:
            return float(self.timer(L, M, m, D, dtype))
        import torch
        from . import Plan, torch_dtype, dtype_code
        key = (L, M, dtype)
        if key not in self._bufs:
            self._bufs.clear()
            td = torch_dtype(dtype_code(dtype))
            self._bufs[key] = (torch.randn(L, dtype=td, device="cuda"), torch.randn(L, dtype=td, device="cuda"),
                               torch.empty(M, dtype=td, device="cuda"))
        f, g, h = self._bufs[key]
        plan = Plan.from_params(L, M, dtype, {"m": m, "D": D, "tile": tile})
        ms = plan.time_convolve(f, g, h, ws=_shared_ws(plan.workspace_bytes), warmup=self.warmup, reps=self.reps)
        plan.close()
        ms.sort()
        return ms[len(ms) // 2]


def a0_candidates(L, M, dtype: str = "c128", batch: int = 1) -> List[dict]:
    """The parameter sets the library's A0 times for a problem, in its order (a
    host-only search with a constant cost)."""
    seen: List[dict] = []

    def t(pr, pm):
        seen.append(params_dict(pm, int(pr.ndim)))
        return 1.0
    run_search(TuneDB(None), L, M, dtype, A0, t, batch)
    return seen


_WS = {"buf": None}


def _shared_ws(nbytes: int):
    """One growing device workspace shared by every timed plan."""
    import torch
    if nbytes == 0:
        return None
    b = _WS["buf"]
    if b is None or b.numel() < nbytes:
        _WS["buf"] = None
        b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _WS["buf"] = b
    return b


def regret(chosen_ms: float, best_ms: float) -> float:
    """T(chosen) / T(exhaustive best) - 1."""
    return chosen_ms / best_ms - 1.0


# ------------------------------------------------------- unequal lengths --

def uneq_key(Lf: int, Lg: int, M: int, dtype: str) -> str:
    return json.dumps({"uneq": [int(Lf), int(Lg)], "M": int(M), "dtype": dtype}, sort_keys=True)


def uneq_candidates(Lf: int, Lg: int, M: int, max_mg: int = 1 << 22, max_pg: int = 4, max_pf: int = 16,
                    d_choices: str = "q") -> List[Tuple[int, int, int]]:
    """(m, Lambda, D) candidates of section 3.5: the longer operand's Lambda m a
    power of two with at most ``max_pg`` blocks (or a single residue), every
    power-of-two Lambda the column stage takes (<= 1024), and the shorter
    operand's m with at most ``max_pf`` blocks."""
    from . import uneq_derive, HdcError
    Ls, Ll = min(Lf, Lg), max(Lf, Lg)
    out = []
    mg = 1
    while mg <= max_mg:
        pg, qg = -(-Ll // mg), -(-M // mg)
        if pg <= max_pg or qg == 1:
            lam = 1
            while lam <= min(1024, mg):
                m = mg // lam
                if -(-Ls // m) <= max_pf:
                    Ds = [qg] + ([1 << i for i in range(20) if (1 << i) < qg] if d_choices == "all" else [])
                    for D in Ds:
                        try:
                            uneq_derive(Lf, Lg, M, m, lam, 1, D)
                        except HdcError:
                            continue
                        out.append((m, lam, D))
                lam *= 2
        mg *= 2
    return out


def _uneq_class(Lf, Lg, M, m, lam):
    """Scale-free class: (p_g, log2 of the shorter operand's m over sqrt(Lambda m))."""
    mg = m * lam
    return (-(-max(Lf, Lg) // mg), int(round(math.log2(m) - math.log2(mg) / 2)))


class TunerUneq:
    """Tunes an unequal-length problem (Lf, Lg, M, dtype) over (m, Lambda, D) on the GPU."""

    def __init__(self, db: Optional[TuneDB] = None, reps: int = 5, warmup: int = 2,
                 timer: Optional[Callable[[int, int, int, int, int, int, str], float]] = None, seed: int = 0):
        self.db = db or TuneDB(None)
        self.reps, self.warmup = reps, warmup
        self.timer = timer  # (Lf, Lg, M, m, lam, D, dtype) -> ms ; defaults to the GPU timer
        self.rng = random.Random(seed)
        self._bufs = {}

    def _gpu_time(self, Lf, Lg, M, m, lam, D, dtype):
        import torch
        from . import UneqPlan, torch_dtype, dtype_code
        key = (Lf, Lg, M, dtype)
        if key not in self._bufs:
            self._bufs.clear()
            td = torch_dtype(dtype_code(dtype))
            self._bufs[key] = (torch.randn(Lf, dtype=td, device="cuda"), torch.randn(Lg, dtype=td, device="cuda"),
                               torch.empty(M, dtype=td, device="cuda"))
        f, g, h = self._bufs[key]
        plan = UneqPlan(Lf, Lg, M, m=m, lam=lam, D=D, dtype=dtype)
        ms = plan.time_convolve(f, g, h, ws=_shared_ws(plan.workspace_bytes), warmup=self.warmup, reps=self.reps)
        plan.close()
        ms.sort()
        return ms[len(ms) // 2]

    def measure(self, Lf, Lg, M, m, lam, D, dtype) -> float:
        if self.timer is not None:
            return float(self.timer(Lf, Lg, M, m, lam, D, dtype))
        return self._gpu_time(Lf, Lg, M, m, lam, D, dtype)

    def _run(self, key, Lf, Lg, M, dtype, cands, table, seen):
        for (m, lam, D) in cands:
            params = {"m": int(m), "lam": int(lam), "D": int(D)}
            pk = json.dumps(params, sort_keys=True)
            if pk in seen:
                continue
            ms = self.measure(Lf, Lg, M, m, lam, D, dtype)
            seen[pk] = ms
            table.append((params, ms))
            self.db.add(key, params, ms)

    @staticmethod
    def _pick(table):
        """argmin; within 1 %: the shorter transform (smaller Lambda m), then the larger Lambda."""
        best = min(ms for _, ms in table)
        near = [(p, ms) for p, ms in table if ms <= best * 1.01]
        near.sort(key=lambda x: (x[0]["m"] * x[0]["lam"], -x[0]["lam"], x[0]["D"], x[1]))
        return near[0]

    def a0(self, Lf: int, Lg: int, M: int, dtype: str = "c128", d_choices: str = "q") -> TuneResult:
        key = uneq_key(Lf, Lg, M, dtype)
        seen = dict(self.db.timings(key))
        table = [(json.loads(pk), ms) for pk, ms in seen.items()]
        self._run(key, Lf, Lg, M, dtype, uneq_candidates(Lf, Lg, M, d_choices=d_choices), table, seen)
        p, ms = self._pick(table)
        return TuneResult(p, ms, table, "A0")

    def a1(self, Lf: int, Lg: int, M: int, dtype: str = "c128", n_random: int = 2, reuse: bool = True) -> TuneResult:
        from . import uneq_derive
        key = uneq_key(Lf, Lg, M, dtype)
        if reuse:
            hit = self.db.best(key)
            if hit is not None:
                return TuneResult(hit[0], hit[1], [hit], "db")
        cands = uneq_candidates(Lf, Lg, M)
        cset = set(cands)
        table: List[Tuple[dict, float]] = []
        seen: Dict[str, float] = {}
        # (1) the derived default; (2) the class of the nearest tuned unequal problem
        s, lg, _ = uneq_derive(Lf, Lg, M, 0, 0, 1, 0)
        seeds = [(s["m"], lg["m"] // s["m"], lg["q"])]
        for cls in self.experience_classes(Lf, Lg, dtype):
            for c in cands:
                if _uneq_class(Lf, Lg, M, c[0], c[1]) == cls and c not in seeds:
                    seeds.append(c)
                    break
        self._run(key, Lf, Lg, M, dtype, seeds, table, seen)
        rest = [c for c in cands if json.dumps({"m": c[0], "lam": c[1], "D": c[2]}, sort_keys=True) not in seen]
        self.rng.shuffle(rest)
        self._run(key, Lf, Lg, M, dtype, rest[:n_random], table, seen)
        # (3) local refinement: Lambda m halved or doubled at the same Lambda, Lambda halved or doubled at the same Lambda m
        for _ in range(4):
            best, _ms = self._pick(table)
            m0, l0 = best["m"], best["lam"]
            neigh = []
            for m, lam in ((m0 // 2, l0), (m0 * 2, l0), (m0 * 2, l0 // 2), (m0 // 2, l0 * 2)):
                for c in cands:
                    if c[0] == m and c[1] == lam and c in cset:
                        neigh.append(c)
                        break
            before = len(table)
            self._run(key, Lf, Lg, M, dtype, neigh, table, seen)
            if len(table) == before:
                break
        p, ms = self._pick(table)
        return TuneResult(p, ms, table, "A1")

    def experience_classes(self, Lf: int, Lg: int, dtype: str, k: int = 2):
        scored = []
        for key in self.db.keys():
            try:
                d = json.loads(key)
            except (ValueError, RecursionError):
                continue
            if not isinstance(d, dict) or "uneq" not in d or d.get("dtype") != dtype:
                continue
            b = self.db.best(key)
            if b is None:
                continue
            try:
                (lf, lg), M = d["uneq"], d["M"]
                dist = abs(math.log2(max(lf, lg)) - math.log2(max(Lf, Lg))) + \
                    abs(math.log2(min(lf, lg)) - math.log2(min(Lf, Lg)))
                scored.append((dist, _uneq_class(lf, lg, M, b[0]["m"], b[0]["lam"])))
            except (KeyError, TypeError, ValueError, ZeroDivisionError):
                continue  # a malformed row
        scored.sort()
        out = []
        for _, c in scored:
            if c not in out:
                out.append(c)
            if len(out) >= k:
                break
        return out


def uneq_nd_candidates(sf, sg, M, axis: int, dtype: str = "c64", max_pg: int = 4):
    """(m, Lambda) candidates of one axis of an unequal-extent N-D problem, the other
    axes at their derived defaults: Lambda m a power of two with at most ``max_pg``
    blocks of the longer operand (or a single residue), Lambda in powers of four."""
    from . import uneq_nd_check, HdcError
    n = len(sf)
    Ll = max(sf[axis], sg[axis])
    out = []
    mg = 1
    while mg <= (1 << 22):
        if -(-Ll // mg) <= max_pg or -(-M[axis] // mg) == 1:
            lam = 1
            while lam <= min(1024, mg):
                m = [0] * n
                ll = [0] * n
                m[axis], ll[axis] = mg // lam, lam
                try:
                    res = uneq_nd_check(sf, sg, M, m, ll, dtype=dtype)
                except HdcError:
                    res = None
                if res is not None and res[axis][1]["N"] <= 4 * M[axis] + 64:
                    out.append((mg // lam, lam))
                lam *= 4
        mg *= 2
    return out


def uneq_nd_separable(sf, sg, M, dtype: str = "c64", timer=None, reps: int = 3, warmup: int = 1):
    """Separable A0 (section 4.2) for an unequal-extent N-D problem: each axis
    searched over its (m, Lambda) candidates with the others at their defaults.
    ``timer(m_list, lam_list) -> ms`` defaults to timing hdc_convolve on the GPU.
    Returns (m per axis, Lambda per axis, number of timings)."""
    n = len(sf)
    if timer is None:
        import torch
        from . import UneqPlan, torch_dtype, dtype_code
        td = torch_dtype(dtype_code(dtype))
        f = torch.randn(tuple(sf), dtype=td, device="cuda")
        g = torch.randn(tuple(sg), dtype=td, device="cuda")
        h = torch.empty(tuple(M), dtype=td, device="cuda")

        def timer(m, lam):
            plan = UneqPlan.nd(sf, sg, M, m=m, lam=lam, dtype=dtype)
            ms = plan.time_convolve(f, g, h, ws=_shared_ws(plan.workspace_bytes), warmup=warmup, reps=reps)
            plan.close()
            ms.sort()
            return ms[len(ms) // 2]
    best_m, best_l, count = [0] * n, [0] * n, 0
    for axis in range(n):
        best = None
        for m, lam in uneq_nd_candidates(sf, sg, M, axis, dtype):
            mm, ll = [0] * n, [0] * n
            mm[axis], ll[axis] = m, lam
            t = timer(mm, ll)
            count += 1
            if best is None or t < best[0]:
                best = (t, m, lam)
        best_m[axis], best_l[axis] = best[1], best[2]
    return best_m, best_l, count


# --------------------------------------------------------------- batches --

def _batch_gpu_time(Ls: Sequence[int], ms: Sequence[int], dtype: str, reps: int = 3, warmup: int = 1) -> float:
    """Median ms of one captured batch over problems Ls with FFT sizes ms (random inputs)."""
    import torch
    from . import Batch, torch_dtype, dtype_code
    B = Batch(Ls, bucket_m=ms, dtype=dtype)
    td = torch_dtype(dtype_code(dtype))
    f = torch.randn(B.total_L, dtype=td, device="cuda")
    g = torch.randn(B.total_L, dtype=td, device="cuda")
    h = torch.empty(B.total_M, dtype=td, device="cuda")
    ws = B.workspace()
    for _ in range(warmup + 1):
        B.convolve(f, g, h, ws=ws)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        B.convolve(f, g, h, ws=ws)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    B.close()
    return sorted(ts)[reps // 2]


def batch_default_m(L: int) -> int:
    """The FFT size hdc_batch_plan gives a problem of length L by default (hdc_batch_default_m)."""
    from ._lib import check, lib
    m = ctypes.c_int64()
    check(lib().hdc_batch_default_m(int(L), ctypes.byref(m)))
    return m.value


def tune_batch(Ls: Sequence[int], dtype: str = "c64", timer: Optional[Callable] = None, max_shift: int = 3,
               reps: int = 3, db: Optional[str] = None, device: Optional[str] = None,
               build: Optional[str] = None) -> Tuple[List[int], Dict[int, List[Tuple[int, float]]]]:
    """Per-bucket exhaustive search (A0 of section 4.2 applied bucket by bucket) for an
    uneven batch with M = 2L - 1.  Problems are grouped by the next power of two of L
    (p = 1); for each group every m = size / 2^j, j = 0 .. max_shift (p = 1, 2, 4, 8),
    and the library's default m (hdc_batch_default_m) are timed on the group's
    problems alone and the fastest kept (ties: the larger m).  ``timer(Ls, ms, dtype) -> ms`` defaults to the captured batch on the
    GPU.  With ``db`` every timing is appended to that JSON-lines database as a bucket
    row (hdc_batch_db_record; ``device`` / ``build`` None: this GPU and library), from
    which ``Batch(..., tune_db=db)`` plans the same choice.  Returns the FFT size of every
    problem and each group's table [(m, ms)]."""
    from . import HdcError, dtype_code
    from ._lib import check, lib
    timer = timer or (lambda ls, ms, dt: _batch_gpu_time(ls, ms, dt, reps=reps))

    def record(size, m, ms):
        if db is not None:
            check(lib().hdc_batch_db_record(db.encode(), size, dtype_code(dtype), m, ms,
                                            device.encode() if device else None, build.encode() if build else None))
    groups: Dict[int, List[int]] = {}
    for i, L in enumerate(Ls):
        groups.setdefault(pow2_ceil(int(L)), []).append(i)
    choice = [batch_default_m(int(L)) for L in Ls]
    tables: Dict[int, List[Tuple[int, float]]] = {}
    for size, idx in sorted(groups.items()):
        gl = [int(Ls[i]) for i in idx]
        rows = []
        cands = [size >> j for j in range(max_shift + 1) if size >> j >= 1]
        dflt = batch_default_m(max(gl))
        if dflt not in cands:
            cands.append(dflt)
        for m in cands:
            try:
                rows.append((m, float(timer(gl, [m] * len(gl), dtype))))
            except HdcError:
                continue
            record(size, m, rows[-1][1])
        tables[size] = rows
        if rows:
            best = min(rows, key=lambda r: (r[1], -r[0]))[0]
            for i in idx:
                choice[i] = best
    return choice, tables


def batch_db_choose(Ls: Sequence[int], dtype: str = "c64", db: Optional[str] = None, Ms: Optional[Sequence[int]] = None,
                    device: Optional[str] = None, build: Optional[str] = None) -> List[int]:
    """The FFT size of every problem that hdc_batch_plan_db takes from ``db``
    (hdc_batch_db_choose, host only; ``device`` / ``build`` None: this GPU and library)."""
    from . import dtype_code
    from ._lib import check, lib
    n = len(Ls)
    arr = ctypes.c_int64 * n
    out = arr()
    check(lib().hdc_batch_db_choose(n, arr(*[int(x) for x in Ls]), arr(*[int(x) for x in Ms]) if Ms is not None else None,
                                    dtype_code(dtype), db.encode() if db else None,
                                    device.encode() if device else None, build.encode() if build else None, out))
    return [int(x) for x in out]
