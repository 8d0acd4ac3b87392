"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the convolution method: it only draws
numbers.  Every array is produced from a numpy PCG64 generator seeded with
``SeedSequence([230610016, cfg, size_idx, which])`` so that any caller can
regenerate exactly the same operands:

* ``which = 0`` draws ``f``, ``which = 1`` draws ``g``, ``which = 2`` draws the
  lengths of a batched workload;
* real and imaginary parts are i.i.d. uniform on [-1, 1], drawn in float64;
* complex64 operands are the float64 draws rounded to complex64, so that a
  float64 consumer given the rounded values sees exactly what the float32
  consumer sees.
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 230610016


def rng(cfg: int, size_idx: int, which: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([ROOT_SEED, int(cfg), int(size_idx), int(which)])))


def uniform_complex(shape, cfg: int, size_idx: int, which: int, dtype=np.complex128) -> np.ndarray:
    """Complex array with re, im ~ U[-1, 1] i.i.d.; ``dtype`` is complex64 or complex128."""
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    r = rng(cfg, size_idx, which)
    n = int(np.prod(shape)) if shape else 1
    re = r.uniform(-1.0, 1.0, n)
    im = r.uniform(-1.0, 1.0, n)
    z = (re + 1j * im).reshape(shape)
    return z.astype(np.dtype(dtype))


def gaussian_integers(shape, bound: int, cfg: int, size_idx: int, which: int) -> np.ndarray:
    """complex128 array whose re and im are integers uniform on [-bound, bound]."""
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    r = rng(cfg, size_idx, which)
    n = int(np.prod(shape))
    re = r.integers(-bound, bound + 1, n).astype(np.float64)
    im = r.integers(-bound, bound + 1, n).astype(np.float64)
    return (re + 1j * im).reshape(shape)


def batch_lengths(n: int, lo_log2: float, hi_log2: float, cfg: int = 3, size_idx: int = 0) -> np.ndarray:
    """``n`` lengths round(2**U[lo_log2, hi_log2]) (log-uniform), as int64."""
    r = rng(cfg, size_idx, 2)
    return np.rint(2.0 ** r.uniform(lo_log2, hi_log2, int(n))).astype(np.int64)


def pair(shape, cfg: int, size_idx: int, dtype=np.complex128):
    """The (f, g) operand pair for one workload entry."""
    return (uniform_complex(shape, cfg, size_idx, 0, dtype),
            uniform_complex(shape, cfg, size_idx, 1, dtype))


def uniform_real(shape, cfg: int, size_idx: int, which: int, dtype=np.float64) -> np.ndarray:
    """Real array ~ U[-1, 1] i.i.d., drawn in float64 and rounded to ``dtype``."""
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    r = rng(cfg, size_idx, which)
    n = int(np.prod(shape)) if shape else 1
    return r.uniform(-1.0, 1.0, n).reshape(shape).astype(np.dtype(dtype))


def integers_real(shape, bound: int, cfg: int, size_idx: int, which: int) -> np.ndarray:
    """float64 array of integers uniform on [-bound, bound]."""
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    r = rng(cfg, size_idx, which)
    return r.integers(-bound, bound + 1, int(np.prod(shape))).astype(np.float64).reshape(shape)
