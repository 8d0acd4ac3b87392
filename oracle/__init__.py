"""CPU FP64 oracle for hybrid dealiased convolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never calls it
and shares no code with it.

The convolution oracle is ``oracle.c`` (plain C, FP64, OpenMP), built into
``liboracle.so`` next to this file by :func:`build`.  It computes the linear
convolution of eq. (5) (section 2.3) two independent ways:

* :func:`direct_1d`, :func:`direct_1d_sampled`, :func:`direct_nd_sampled` --
  the defining sum; :func:`direct_1d_real` the same sum in real arithmetic for
  real operands (the real case section 7 leaves to future work);
  :func:`direct_multi` and :func:`padded_multi` the convolution of A >= 2
  sequences (section 6.1's multi-convolution), by the defining sum applied
  operand by operand and by explicit padding;
* :func:`padded_1d`, :func:`padded_nd` -- explicit dealiasing (section 3.1):
  zero padding to the smallest 2^a 3^b 5^c 7^d size >= 2L-1, DFT with
  zeta = e^{+2 pi i/n}, product, inverse DFT with 1/n, crop to M.

:func:`padded_dft` is the zero-extended forward DFT whose entries the residues
of eq. (3) (section 2.2) enumerate.  ``mlp.py`` holds the FP64 reference of
the parameter predictor's network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_direct_1d.argtypes = [_I64, _I64, _I64, _P, _P, _P]
        lib.oracle_direct_1d_sampled.argtypes = [_I64, _I64, _P, _P, _P, _I64, _P]
        lib.oracle_direct_nd_sampled.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _I64, _P]
        lib.oracle_padded_1d.argtypes = [_I64, _I64, _I64, _P, _P, _P]
        lib.oracle_direct_1d_uneq.argtypes = [_I64, _I64, _I64, _I64, _P, _P, _P]
        lib.oracle_direct_1d_uneq_sampled.argtypes = [_I64, _I64, _I64, _P, _P, _P, _I64, _P]
        lib.oracle_direct_1d_real.argtypes = [_I64, _I64, _I64, _P, _P, _P]
        lib.oracle_padded_1d_uneq.argtypes = [_I64, _I64, _I64, _I64, _P, _P, _P]
        lib.oracle_padded_nd.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P]
        lib.oracle_direct_nd_uneq_sampled.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P, _I64, _P]
        lib.oracle_padded_nd_uneq.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P]
        lib.oracle_dft.argtypes = [_I64, _P, ctypes.c_int]
        lib.oracle_padded_dft.argtypes = [_I64, _I64, _P, _P]
        lib.oracle_friendly_size.argtypes = [_I64]
        lib.oracle_friendly_size.restype = _I64
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _as_2d(x):
    x = _c128(x)
    if x.ndim == 1:
        return x.reshape(-1, 1), True
    if x.ndim != 2:
        raise ValueError("1D oracle takes (L,) or (L, C) arrays")
    return x, False


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def friendly_size(n: int) -> int:
    """Smallest 2^a 3^b 5^c 7^d >= n."""
    return int(_load().oracle_friendly_size(int(n)))


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name}: invalid arguments")


def direct_1d(f, g, M: int) -> np.ndarray:
    """h_k = sum_j f_j g_{k-j} for k < M (eq. (5)); f of shape (Lf,) or (Lf, C), g of
    shape (Lg,) or (Lg, C) (Lf and Lg may differ: the unequal case of section 3.5)."""
    f2, flat = _as_2d(f)
    g2, _ = _as_2d(g)
    if f2.shape[1] != g2.shape[1]:
        raise ValueError("f and g must have the same number of copies")
    Lf, C = f2.shape
    h = np.empty((int(M), C), np.complex128)
    _check(_load().oracle_direct_1d_uneq(Lf, g2.shape[0], int(M), C, f2.ctypes.data, g2.ctypes.data, h.ctypes.data),
           "direct_1d")
    return h.reshape(-1) if flat else h


def direct_1d_real(f, g, M: int) -> np.ndarray:
    """eq. (5) for real f, g of shape (L,) or (L, C), in real FP64 arithmetic."""
    f2 = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    g2 = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    flat = f2.ndim == 1
    f2, g2 = f2.reshape(f2.shape[0], -1), g2.reshape(g2.shape[0], -1)
    if f2.shape != g2.shape:
        raise ValueError("f and g must have the same shape")
    L, C = f2.shape
    h = np.empty((int(M), C), np.float64)
    _check(_load().oracle_direct_1d_real(L, int(M), C, f2.ctypes.data, g2.ctypes.data, h.ctypes.data),
           "direct_1d_real")
    return h.reshape(-1) if flat else h


def direct_1d_sampled(f, g, ks) -> np.ndarray:
    """eq. (5) evaluated only at the output indices ``ks`` (f and g may differ in length)."""
    f2, flat = _as_2d(f)
    g2, _ = _as_2d(g)
    if f2.shape[1] != g2.shape[1]:
        raise ValueError("f and g must have the same number of copies")
    Lf, C = f2.shape
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.empty((ks.size, C), np.complex128)
    _check(_load().oracle_direct_1d_uneq_sampled(Lf, g2.shape[0], C, f2.ctypes.data, g2.ctypes.data, ks.ctypes.data,
                                                 ks.size, out.ctypes.data), "direct_1d_sampled")
    return out.reshape(-1) if flat else out


def direct_nd_sampled(f, g, M, ks) -> np.ndarray:
    """N-D eq. (5) at the row-major linear indices ``ks`` of the output box M; f and
    g may have different extents (same number of axes)."""
    f = _c128(f)
    g = _c128(g)
    nd = f.ndim
    if g.ndim != nd:
        raise ValueError("f and g must have the same number of axes")
    Lf = np.ascontiguousarray(f.shape, dtype=np.int64)
    Lg = np.ascontiguousarray(g.shape, dtype=np.int64)
    Ms = np.ascontiguousarray(M, dtype=np.int64)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.empty(ks.size, np.complex128)
    _check(_load().oracle_direct_nd_uneq_sampled(nd, Lf.ctypes.data, Lg.ctypes.data, Ms.ctypes.data, f.ctypes.data,
                                                 g.ctypes.data, ks.ctypes.data, ks.size, out.ctypes.data),
           "direct_nd_sampled")
    return out


def direct_nd(f, g, M) -> np.ndarray:
    """N-D eq. (5) over the whole output box (small problems only)."""
    M = tuple(int(x) for x in M)
    ks = np.arange(int(np.prod(M)), dtype=np.int64)
    return direct_nd_sampled(f, g, M, ks).reshape(M)


def padded_1d(f, g, M: int) -> np.ndarray:
    """Explicitly zero-padded FFT convolution (section 3.1), output length M; f and g may
    have different lengths (padding to the smallest friendly size >= Lf + Lg - 1)."""
    f2, flat = _as_2d(f)
    g2, _ = _as_2d(g)
    if f2.shape[1] != g2.shape[1]:
        raise ValueError("f and g must have the same number of copies")
    Lf, C = f2.shape
    h = np.empty((int(M), C), np.complex128)
    _check(_load().oracle_padded_1d_uneq(Lf, g2.shape[0], int(M), C, f2.ctypes.data, g2.ctypes.data, h.ctypes.data),
           "padded_1d")
    return h.reshape(-1) if flat else h


def padded_nd(f, g, M) -> np.ndarray:
    """Explicitly zero-padded FFT convolution in 1..3 dimensions (f and g may differ
    in extent along any axis)."""
    f = _c128(f)
    g = _c128(g)
    if g.ndim != f.ndim:
        raise ValueError("f and g must have the same number of axes")
    Lf = np.ascontiguousarray(f.shape, dtype=np.int64)
    Lg = np.ascontiguousarray(g.shape, dtype=np.int64)
    Ms = np.ascontiguousarray(M, dtype=np.int64)
    h = np.empty(tuple(int(x) for x in M), np.complex128)
    _check(_load().oracle_padded_nd_uneq(f.ndim, Lf.ctypes.data, Lg.ctypes.data, Ms.ctypes.data, f.ctypes.data,
                                         g.ctypes.data, h.ctypes.data), "padded_nd")
    return h


def dft(x, sign: int) -> np.ndarray:
    """X_k = sum_j exp(sign 2 pi i k j / n) x_j (unscaled)."""
    y = _c128(x).copy()
    _check(_load().oracle_dft(y.size, y.ctypes.data, int(sign)), "dft")
    return y


def padded_dft(x, N: int) -> np.ndarray:
    """X_k = sum_{j<L} zeta_N^{+kj} x_j, k < N (the zero-extended forward transform)."""
    x = _c128(x)
    X = np.empty(int(N), np.complex128)
    _check(_load().oracle_padded_dft(x.size, int(N), x.ctypes.data, X.ctypes.data), "padded_dft")
    return X


def direct_multi(xs, M: int) -> np.ndarray:
    """The convolution of A >= 2 sequences (section 6.1's multi-convolution of N arrays):
    h_k = sum over j_0 + ... + j_{A-1} = k of prod_a x_a[j_a], k < M; x_a of shape (L_a,)
    or (L_a, C).  Evaluated as the defining sum of eq. (5) applied operand by operand
    (the nested sums regroup the A-fold sum exactly)."""
    flat = np.asarray(xs[0]).ndim == 1
    xs = [_as_2d(x)[0] for x in xs]
    if len(xs) < 2:
        raise ValueError("need at least two sequences")
    h = xs[0]
    for x in xs[1:]:
        h = direct_1d(h, x, h.shape[0] + x.shape[0] - 1)
        h = h.reshape(-1, x.shape[1])
    out = np.zeros((int(M), h.shape[1]), np.complex128)
    n = min(int(M), h.shape[0])
    out[:n] = h[:n]
    return out.reshape(-1) if flat else out


def padded_multi(xs, M: int) -> np.ndarray:
    """Explicit dealiasing for A sequences (section 3.1 applied to section 6.1's N arrays):
    zero-pad every x_a to the smallest friendly size Ne >= sum_a L_a - (A - 1), take their
    DFTs, multiply them pointwise, inverse DFT with 1/Ne, crop to M (zeros beyond)."""
    flat = np.asarray(xs[0]).ndim == 1
    xs = [_as_2d(x)[0] for x in xs]
    C = xs[0].shape[1]
    K = sum(x.shape[0] for x in xs) - (len(xs) - 1)
    Ne = friendly_size(K)
    out = np.zeros((int(M), C), np.complex128)
    for c in range(C):
        H = np.ones(Ne, np.complex128)
        for x in xs:
            z = np.zeros(Ne, np.complex128)
            z[:x.shape[0]] = x[:, c]
            H *= dft(z, +1)
        h = dft(H, -1) / Ne
        n = min(int(M), K)
        out[:n, c] = h[:n]
    return out.reshape(-1) if flat else out


def multi_sampled(xs, ks) -> np.ndarray:
    """Outputs ks of the A-fold convolution: the first A - 1 operands by padded_multi (or
    the single first operand), the last one by the defining sum at each k."""
    flat = np.asarray(xs[0]).ndim == 1
    xs = [_as_2d(x)[0] for x in xs]
    pre = xs[0] if len(xs) == 2 else padded_multi(xs[:-1], sum(x.shape[0] for x in xs[:-1]) - (len(xs) - 2))
    out = direct_1d_sampled(pre, xs[-1], ks)
    return out.reshape(-1) if flat else out


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 over all entries (b is the reference)."""
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)
