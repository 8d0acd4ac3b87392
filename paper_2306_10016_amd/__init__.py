"""Python binding of libhdc (hybrid dealiased convolution on MI355X / gfx950).

Argument marshalling only: every step of the convolution runs in the HIP
kernels of ``libhdc.so``; PyTorch supplies device memory and streams.  There
is no CPU fallback: if the shared library is missing, importing the binding
raises.

Names follow ``include/hdc.h``:

* :class:`Plan` wraps ``hdc_plan`` / ``hdc_plan_nd`` and exposes
  ``convolve`` (``hdc_convolve``), ``forward``, ``multiply``, ``backward`` and
  ``residues_natural``;
* :class:`Batch` wraps ``hdc_batch_*`` (uneven-length batches, replayed
  from a captured HIP graph);
* :class:`UneqPlan` wraps ``hdc_plan_uneq`` (operands of different lengths,
  section 3.5) and adds ``forward_operand`` (``hdc_forward_operand``);
* :class:`MultiPlan` wraps ``hdc_plan_multi`` / ``hdc_convolve_multi`` (the
  convolution of A sequences, section 6.1);
* :func:`derive` / :func:`uneq_derive` are the host-only admissibility checks
  (``hdc_derive`` / ``hdc_uneq_derive``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

from . import _lib
from ._lib import AxisDesc, HdcError, lib, check  # noqa: F401

C64, C128, R32, R64 = 0, 1, 2, 3
# bytes of the per-GPU device array that hdc_convolve_noalloc uses as its workspace
SCRATCH_BYTES = 64 << 20
_DT = {"c64": C64, "complex64": C64, "c128": C128, "complex128": C128, "r32": R32, "float32": R32,
       "r64": R64, "float64": R64, C64: C64, C128: C128, R32: R32, R64: R64}


def dtype_code(dtype) -> int:
    if hasattr(dtype, "is_complex"):  # torch dtype
        import torch
        return {torch.complex128: C128, torch.complex64: C64, torch.float64: R64, torch.float32: R32}[dtype]
    return _DT[dtype]


def torch_dtype(code: int):
    import torch
    return {C128: torch.complex128, C64: torch.complex64, R64: torch.float64, R32: torch.float32}[code]


def is_real(code: int) -> bool:
    return code in (R32, R64)


def derive(L: int, M: int, m: int, p: int = 0, q: int = 0, C: int = 1, D: int = 0, dtype="c128") -> dict:
    """Admissibility and derived parameters (no device is touched)."""
    d = AxisDesc()
    check(lib().hdc_derive(L, M, m, p, q, C, D, dtype_code(dtype), ctypes.byref(d)))
    return d.as_dict()


def check_nd(L, M, m, p=None, q=None, D=None, dtype="c64"):
    """Host-only validation of an N-D plan (hdc_plan_nd_check); returns the axis descriptions."""
    n = len(L)
    arr = ctypes.c_int64 * n

    def a(v):
        return arr(*[int(x) for x in v]) if v is not None else None
    out = (AxisDesc * n)()
    check(lib().hdc_plan_nd_check(n, a(L), a(M), a(m), a(p), a(q), a(D), dtype_code(dtype), out))
    return [d.as_dict() for d in out]


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, dtype_code_, numel: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch_dtype(dtype_code_):
        raise TypeError(f"{name} has dtype {t.dtype}, plan expects {torch_dtype(dtype_code_)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


class Plan:
    """A 1D (``Plan(L, M, m, ...)``) or N-D (``Plan.nd(...)``) hybrid-dealiasing plan."""

    def __init__(self, L: int, M: int, m: int, p: int = 0, q: int = 0, C: int = 1, D: int = 0, dtype="c128",
                 _handle=None):
        self._lib = lib()
        if _handle is None:
            h = ctypes.c_void_p()
            check(self._lib.hdc_plan(ctypes.byref(h), int(L), int(M), int(m), int(p), int(q), int(C), int(D),
                                     dtype_code(dtype)))
            _handle = h
        self._h = _handle
        self.dtype = dtype_code(dtype)
        nd = ctypes.c_int()
        self.axes = []
        check(self._lib.hdc_plan_axis(self._h, 0, ctypes.byref(nd), None))
        self.ndim = nd.value
        for a in range(self.ndim):
            d = AxisDesc()
            check(self._lib.hdc_plan_axis(self._h, a, None, ctypes.byref(d)))
            self.axes.append(d.as_dict())
        sz = ctypes.c_size_t()
        check(self._lib.hdc_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = sz.value
        self._ws = None

    @classmethod
    def nd(cls, L: Sequence[int], M: Sequence[int], m: Sequence[int], p=None, q=None, D=None, dtype="c64"):
        n = len(L)
        arr = ctypes.c_int64 * n

        def a(v):
            return arr(*[int(x) for x in v]) if v is not None else None
        h = ctypes.c_void_p()
        check(lib().hdc_plan_nd(ctypes.byref(h), n, a(L), a(M), a(m), a(p), a(q), a(D), dtype_code(dtype)))
        return cls(0, 0, 0, dtype=dtype, _handle=h)

    @classmethod
    def from_params(cls, L, M, dtype, params: dict, batch: int = 1):
        """Plan from a tuner's parameter set (hdc_plan_params): ``params`` holds "m" and
        "D" (and optionally "tile", 0 = default), scalars for 1D (int L) or per-axis
        lists for N-D; p and q are derived."""
        from ._lib import Params
        from .tune import problem
        pr = problem(L, M, dtype, batch)
        nd = pr.ndim
        pm = Params()

        def axis(v, a):
            return int(v[a]) if isinstance(v, (list, tuple)) else int(v)
        for a in range(nd):
            pm.m[a] = axis(params["m"], a)
            pm.D[a] = axis(params.get("D", 0), a)
            pm.tile[a] = axis(params.get("tile", 0), a)
        h = ctypes.c_void_p()
        check(lib().hdc_plan_params(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(pm)))
        return cls(0, 0, 0, dtype=dtype, _handle=h)

    # -- properties
    @property
    def L(self):
        return tuple(ax["L"] for ax in self.axes) if self.ndim > 1 else self.axes[0]["L"]

    @property
    def M(self):
        return tuple(ax["M"] for ax in self.axes) if self.ndim > 1 else self.axes[0]["M"]

    @property
    def C(self) -> int:
        return self.axes[0]["C"]

    def in_numel(self) -> int:
        n = 1
        for ax in self.axes:
            n *= ax["L"]
        return n * (self.C if self.ndim == 1 else 1)

    def out_numel(self) -> int:
        n = 1
        for ax in self.axes:
            n *= ax["M"]
        return n * (self.C if self.ndim == 1 else 1)

    def out_shape(self):
        if self.ndim == 1:
            return (self.axes[0]["M"],) if self.C == 1 else (self.axes[0]["M"], self.C)
        return tuple(ax["M"] for ax in self.axes)

    def workspace(self, device=None):
        """A cached device workspace of ``workspace_bytes`` (allocated by torch).  Calls
        that use it must not overlap: concurrent calls on different streams each
        pass a workspace of their own (``ws=``)."""
        import torch
        if self.workspace_bytes == 0:
            return None
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def residue_buffer(self, device=None):
        import torch
        sz = ctypes.c_size_t()
        check(self._lib.hdc_residue_buffer_size(self._h, ctypes.byref(sz)))
        esz = 16 if self.dtype == C128 else 8
        return torch.empty(sz.value // esz, dtype=torch_dtype(self.dtype), device=device or "cuda")

    # -- execution
    def convolve(self, f, g, out=None, ws=None, stream=None):
        """h = f * g (hdc_convolve); returns ``out`` (allocated if None)."""
        import torch
        _check_tensor(f, self.dtype, self.in_numel(), "f")
        _check_tensor(g, self.dtype, self.in_numel(), "g")
        if out is None:
            out = torch.empty(self.out_shape(), dtype=torch_dtype(self.dtype), device=f.device)
        _check_tensor(out, self.dtype, self.out_numel(), "out")
        if ws is None:
            ws = self.workspace(f.device)
        check(self._lib.hdc_convolve(self._h, _ptr(f), _ptr(g), _ptr(out),
                                     _ptr(ws) if ws is not None else None, _stream(stream)))
        return out

    def convolve_noalloc(self, f, g, out, stream=None):
        """h = f * g through hdc_convolve_noalloc: the library's per-GPU scratch array
        serves as the workspace, so the call allocates nothing (``out`` is required)."""
        _check_tensor(f, self.dtype, self.in_numel(), "f")
        _check_tensor(g, self.dtype, self.in_numel(), "g")
        _check_tensor(out, self.dtype, self.out_numel(), "out")
        check(self._lib.hdc_convolve_noalloc(self._h, _ptr(f), _ptr(g), _ptr(out), _stream(stream)))
        return out

    def forward(self, f, F, r0: int, stream=None):
        _check_tensor(f, self.dtype, self.in_numel(), "f")
        check(self._lib.hdc_forward(self._h, _ptr(f), _ptr(F), int(r0), None, _stream(stream)))
        return F

    def multiply(self, F, G, r0: int, stream=None):
        check(self._lib.hdc_multiply(self._h, _ptr(F), _ptr(G), int(r0), _stream(stream)))
        return F

    def backward(self, F, h, r0: int, stream=None):
        _check_tensor(h, self.dtype, self.out_numel(), "h")
        check(self._lib.hdc_backward(self._h, _ptr(F), _ptr(h), int(r0), None, _stream(stream)))
        return h

    def residues_natural(self, F, r0: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(F)
        check(self._lib.hdc_residues_natural(self._h, _ptr(F), int(r0), _ptr(out), _stream(stream)))
        return out

    def time_convolve(self, f, g, out, ws=None, warmup: int = 2, reps: int = 5, stream=None):
        """Per-repetition milliseconds from hdc_time_convolve (HIP events)."""
        ms = (ctypes.c_float * reps)()
        if ws is None:
            ws = self.workspace(f.device)
        check(self._lib.hdc_time_convolve(self._h, _ptr(f), _ptr(g), _ptr(out),
                                          _ptr(ws) if ws is not None else None, _stream(stream),
                                          int(warmup), int(reps), ms))
        return list(ms)

    KIND_NAMES = ("fused", "col_fwd", "row", "col_bwd", "row_raw", "qsum", "rowconv", "real_scale")

    def convolve_profiled(self, f, g, out, ws=None, stream=None, max_launches: int = 4096):
        """hdc_convolve with per-launch HIP-event timing: list of (kind, ms, algorithmic bytes)."""
        n = ctypes.c_int()
        kinds = (ctypes.c_int32 * max_launches)()
        ms = (ctypes.c_float * max_launches)()
        by = (ctypes.c_double * max_launches)()
        if ws is None:
            ws = self.workspace(f.device)
        check(self._lib.hdc_convolve_profiled(self._h, _ptr(f), _ptr(g), _ptr(out),
                                              _ptr(ws) if ws is not None else None, _stream(stream),
                                              max_launches, ctypes.byref(n), kinds, ms, by))
        k = min(n.value, max_launches)
        return [(self.KIND_NAMES[kinds[i]], ms[i], by[i]) for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def uneq_derive(Lf: int, Lg: int, M: int, m: int = 0, lam: int = 0, C: int = 1, D: int = 0, dtype="c128"):
    """Host-only derivation of an unequal-length plan (hdc_uneq_derive):
    (shorter operand's description, longer operand's description, swapped)."""
    s, lg, sw = AxisDesc(), AxisDesc(), ctypes.c_int()
    check(lib().hdc_uneq_derive(int(Lf), int(Lg), int(M), int(m), int(lam), int(C), int(D), dtype_code(dtype),
                                ctypes.byref(s), ctypes.byref(lg), ctypes.byref(sw)))
    return s.as_dict(), lg.as_dict(), bool(sw.value)


def uneq_nd_check(Lf, Lg, M=None, m=None, lam=None, D=None, dtype="c64"):
    """Host-only check of an unequal-extent N-D plan (hdc_uneq_nd_check):
    per axis (shorter operand's description, longer operand's, f is the longer)."""
    n = len(Lf)
    arr = ctypes.c_int64 * n
    M = [int(a) + int(b) - 1 for a, b in zip(Lf, Lg)] if M is None else M

    def a(v):
        return arr(*[int(x) for x in v]) if v is not None else None
    so, lo, sw = (AxisDesc * n)(), (AxisDesc * n)(), (ctypes.c_int * n)()
    check(lib().hdc_uneq_nd_check(n, a(Lf), a(Lg), a(M), a(m), a(lam), a(D), dtype_code(dtype), so, lo, sw))
    return [(so[i].as_dict(), lo[i].as_dict(), bool(sw[i])) for i in range(n)]


class UneqPlan(Plan):
    """Unequal operand lengths (hdc_plan_uneq, section 3.5): f of length Lf, g of
    length Lg, output length M >= Lf + Lg - 1; the shorter operand uses m-point
    residues and the longer Lambda m-point ones.  ``axes[a]`` describes the
    longer operand on axis a (the geometry of the product and the backward),
    ``short_axes[a]`` the shorter one (``short_axis`` for 1D).  ``UneqPlan.nd``
    builds the 2D/3D form (hdc_plan_uneq_nd)."""

    def __init__(self, Lf: int, Lg: int, M: Optional[int] = None, m: int = 0, lam: int = 0, C: int = 1, D: int = 0,
                 dtype="c128", _handle=None, _shapes=None):
        if _handle is None:
            M = int(Lf) + int(Lg) - 1 if M is None else int(M)
            h = ctypes.c_void_p()
            check(lib().hdc_plan_uneq(ctypes.byref(h), int(Lf), int(Lg), M, int(m), int(lam), int(C), int(D),
                                      dtype_code(dtype)))
            _handle = h
            _shapes = ((int(Lf),), (int(Lg),))
        super().__init__(0, 0, 0, dtype=dtype, _handle=_handle)
        self.short_axes = []
        for a in range(self.ndim):
            d = AxisDesc()
            check(self._lib.hdc_plan_axis(self._h, self.ndim + a, None, ctypes.byref(d)))
            self.short_axes.append(d.as_dict())
        self.short_axis = self.short_axes[0]
        self.f_shape, self.g_shape = _shapes
        if self.ndim == 1:
            self.Lf, self.Lg = self.f_shape[0], self.g_shape[0]
        self.lams = [ax["m"] // sa["m"] for ax, sa in zip(self.axes, self.short_axes)]
        self.lam = self.lams[0]

    @classmethod
    def nd(cls, Lf: Sequence[int], Lg: Sequence[int], M: Optional[Sequence[int]] = None, m=None, lam=None, D=None,
           dtype="c64"):
        n = len(Lf)
        arr = ctypes.c_int64 * n
        M = [int(a) + int(b) - 1 for a, b in zip(Lf, Lg)] if M is None else M

        def a(v):
            return arr(*[int(x) for x in v]) if v is not None else None
        h = ctypes.c_void_p()
        check(lib().hdc_plan_uneq_nd(ctypes.byref(h), n, a(Lf), a(Lg), a(M), a(m), a(lam), a(D), dtype_code(dtype)))
        return cls(0, 0, dtype=dtype, _handle=h, _shapes=(tuple(int(x) for x in Lf), tuple(int(x) for x in Lg)))

    @property
    def L(self):
        return (self.f_shape, self.g_shape) if self.ndim > 1 else (self.Lf, self.Lg)

    def _numel(self, shape):
        n = 1
        for x in shape:
            n *= x
        return n * (self.C if self.ndim == 1 else 1)

    def convolve(self, f, g, out=None, ws=None, stream=None):
        """h = f * g (hdc_convolve of the unequal-length plan)."""
        import torch
        _check_tensor(f, self.dtype, self._numel(self.f_shape), "f")
        _check_tensor(g, self.dtype, self._numel(self.g_shape), "g")
        if out is None:
            out = torch.empty(self.out_shape(), dtype=torch_dtype(self.dtype), device=f.device)
        _check_tensor(out, self.dtype, self.out_numel(), "out")
        if ws is None:
            ws = self.workspace(f.device)
        check(self._lib.hdc_convolve(self._h, _ptr(f), _ptr(g), _ptr(out),
                                     _ptr(ws) if ws is not None else None, _stream(stream)))
        return out

    def convolve_noalloc(self, f, g, out, stream=None):
        """hdc_convolve_noalloc of the unequal-length plan (library scratch as workspace)."""
        _check_tensor(f, self.dtype, self._numel(self.f_shape), "f")
        _check_tensor(g, self.dtype, self._numel(self.g_shape), "g")
        _check_tensor(out, self.dtype, self.out_numel(), "out")
        check(self._lib.hdc_convolve_noalloc(self._h, _ptr(f), _ptr(g), _ptr(out), _stream(stream)))
        return out

    def forward_operand(self, operand: int, x, F, r0: int, stream=None):
        """hdc_forward_operand: residues of group r0 of f (operand 0) or g (operand 1),
        in the longer operand's geometry."""
        _check_tensor(x, self.dtype, self._numel(self.f_shape if operand == 0 else self.g_shape), "x")
        check(self._lib.hdc_forward_operand(self._h, int(operand), _ptr(x), _ptr(F), int(r0), None, _stream(stream)))
        return F

    def forward(self, f, F, r0: int, stream=None):
        raise HdcError(1, "unequal-length plan: use forward_operand")


class MultiPlan(Plan):
    """Multi-convolution (hdc_plan_multi, section 6.1): h = x_0 * ... * x_{A-1} for
    A = 2 .. 8 sequences of length L (C copies), output length M (default the
    A(L-1)+1 terms of the linear result)."""

    def __init__(self, A: int, L: int, M: Optional[int] = None, m: int = 0, p: int = 0, q: int = 0, C: int = 1,
                 D: int = 0, dtype="c128"):
        M = int(A) * (int(L) - 1) + 1 if M is None else int(M)
        h = ctypes.c_void_p()
        check(lib().hdc_plan_multi(ctypes.byref(h), int(A), int(L), M, int(m), int(p), int(q), int(C), int(D),
                                   dtype_code(dtype)))
        super().__init__(0, 0, 0, dtype=dtype, _handle=h)
        self.A = int(A)

    @classmethod
    def nd(cls, A: int, L: Sequence[int], M: Optional[Sequence[int]] = None, m: Optional[Sequence[int]] = None,
           D: Optional[Sequence[int]] = None, dtype="c64"):
        """2D/3D multi-convolution (hdc_plan_multi_nd): A operands of the box L, output box
        M (default the A(L-1)+1 terms per axis); m defaults to the power of two >= L per
        axis (at most 2^20 on outer axes)."""
        n = len(L)
        M = [int(A) * (int(x) - 1) + 1 for x in L] if M is None else [int(x) for x in M]
        if m is None:
            m = []
            for a, x in enumerate(L):
                v = 1
                while v < int(x):
                    v <<= 1
                m.append(min(v, 1 << 20) if a < n - 1 else v)
        arr = ctypes.c_int64 * n
        h = ctypes.c_void_p()
        check(lib().hdc_plan_multi_nd(ctypes.byref(h), int(A), n, arr(*[int(x) for x in L]), arr(*M),
                                      arr(*[int(x) for x in m]), arr(*[int(x) for x in D]) if D else None,
                                      dtype_code(dtype)))
        obj = cls.__new__(cls)
        Plan.__init__(obj, 0, 0, 0, dtype=dtype, _handle=h)
        obj.A = int(A)
        return obj

    def convolve(self, xs, out=None, ws=None, stream=None):
        """h = x_0 * ... * x_{A-1} (hdc_convolve_multi); ``xs`` holds the A device tensors."""
        import torch
        if len(xs) != self.A:
            raise ValueError(f"plan has {self.A} operands, got {len(xs)}")
        for i, x in enumerate(xs):
            _check_tensor(x, self.dtype, self.in_numel(), f"x[{i}]")
        if out is None:
            out = torch.empty(self.out_shape(), dtype=torch_dtype(self.dtype), device=xs[0].device)
        _check_tensor(out, self.dtype, self.out_numel(), "out")
        if ws is None:
            ws = self.workspace(xs[0].device)
        arr = (ctypes.c_void_p * self.A)(*[x.data_ptr() for x in xs])
        check(self._lib.hdc_convolve_multi(self._h, arr, _ptr(out), _ptr(ws) if ws is not None else None,
                                           _stream(stream)))
        return out


class Profile:
    """Context manager around hdc_profile_begin/end: per-launch (kind, ms, bytes) of one plan."""

    def __init__(self, plan: Optional[Plan] = None, max_launches: int = 1 << 16):
        self.plan = plan
        self.max = max_launches
        self.launches = []

    def __enter__(self):
        check(lib().hdc_profile_begin(self.plan._h if self.plan is not None else None))
        return self

    def __exit__(self, *exc):
        n = ctypes.c_int()
        kinds = (ctypes.c_int32 * self.max)()
        ms = (ctypes.c_float * self.max)()
        by = (ctypes.c_double * self.max)()
        check(lib().hdc_profile_end(self.max, ctypes.byref(n), kinds, ms, by))
        k = min(n.value, self.max)
        self.launches = [(Plan.KIND_NAMES[kinds[i]], ms[i], by[i]) for i in range(k)]
        return False

    def summary(self) -> dict:
        """Per kernel kind: launches, total ms, mean ms, mean algorithmic bytes, GB/s."""
        out = {}
        for kind, ms, by in self.launches:
            d = out.setdefault(kind, {"launches": 0, "ms": 0.0, "bytes": 0.0})
            d["launches"] += 1
            d["ms"] += ms
            d["bytes"] += by
        for d in out.values():
            d["mean_ms"] = d["ms"] / d["launches"]
            d["mean_bytes"] = d["bytes"] / d["launches"]
            d["GBps"] = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        return out


class Batch:
    """Uneven-length batch of 1D convolutions packed back to back (hdc_batch_plan; with
    ``tune_db``, hdc_batch_plan_db: each bucket's FFT size from the fastest row that
    ``tune.tune_batch(..., db=tune_db)`` recorded on this device and build)."""

    def __init__(self, L: Sequence[int], M: Optional[Sequence[int]] = None, bucket_m: Optional[Sequence[int]] = None,
                 dtype="c64", tune_db: Optional[str] = None):
        self._lib = lib()
        n = len(L)
        arr = ctypes.c_int64 * n
        self.L = [int(x) for x in L]
        self.M = [int(x) for x in M] if M is not None else [2 * x - 1 for x in self.L]
        h = ctypes.c_void_p()
        if tune_db is not None:
            if bucket_m is not None:
                raise ValueError("give bucket_m or tune_db, not both")
            check(self._lib.hdc_batch_plan_db(ctypes.byref(h), n, arr(*self.L), arr(*self.M), dtype_code(dtype),
                                              tune_db.encode()))
        else:
            check(self._lib.hdc_batch_plan(ctypes.byref(h), n, arr(*self.L), arr(*self.M),
                                           arr(*[int(x) for x in bucket_m]) if bucket_m is not None else None,
                                           dtype_code(dtype)))
        self._h = h
        self.dtype = dtype_code(dtype)
        sz = ctypes.c_size_t()
        check(self._lib.hdc_batch_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = sz.value
        nb, tl, tm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(self._lib.hdc_batch_info(self._h, ctypes.byref(nb), ctypes.byref(tl), ctypes.byref(tm)))
        self.n_buckets, self.total_L, self.total_M = nb.value, tl.value, tm.value
        self._ws = None

    def workspace(self, device=None):
        import torch
        if self.workspace_bytes == 0:
            return None
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def convolve(self, f, g, out=None, ws=None, stream=None, graph: bool = True):
        import torch
        _check_tensor(f, self.dtype, self.total_L, "f")
        _check_tensor(g, self.dtype, self.total_L, "g")
        if out is None:
            out = torch.empty(self.total_M, dtype=torch_dtype(self.dtype), device=f.device)
        _check_tensor(out, self.dtype, self.total_M, "out")
        if ws is None:
            ws = self.workspace(f.device)
        fn = self._lib.hdc_batch_convolve if graph else self._lib.hdc_batch_convolve_eager
        check(fn(self._h, _ptr(f), _ptr(g), _ptr(out), _ptr(ws) if ws is not None else None, _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
