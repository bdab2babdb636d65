"""Seeded synthetic inputs shaped like the paper's workloads (input generation only).

Holds token-set transcriptions (``tokensets``) and corpus generators (``gen.c``, loaded
through ctypes).  Nothing here lexes or certifies: both the library's benchmarks and the
oracle's tests draw their inputs from this module, and it imports neither of them.

Corpora (all deterministic from their seed):
  * ``clike(n, seed, bcomment=False)`` -- lines of Poisson(8) C-like tokens (IDENT .35,
    INT .15, OP .25, STR .05, LCOMMENT .05; + BCOMMENT .05 when ``bcomment``), 1-4 space/tab
    separators, newline-terminated, tail padded with newlines;
  * ``json(n, seed)`` -- pretty-printed nested objects/arrays (2-space indent, depth <= 6,
    keys of 3-12 letters, values 40% string / 30% number / 10% keyword / 20% nested);
  * ``loglines(n, period)`` -- the planning workload: a newline at every offset that is
    period-1 modulo period, other bytes 'x';
  * ``docs(count, seed)`` -- the batched-documents workload (log-normal sizes, token-set mix);
  * ``lognormal_sizes``, ``uniform``, ``exponential`` -- scalar draws for the serving loop.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import tokensets  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-o", _LIB_PATH,
           os.path.join(_HERE, "gen.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        P, U64, D = C.c_void_p, C.c_uint64, C.c_double
        lib.wl_clike.argtypes = [P, U64, U64, C.c_int, U64]
        lib.wl_json.argtypes = [P, U64, U64]
        lib.wl_lognormal_sizes.argtypes = [P, U64, D, D, U64, U64, U64]
        lib.wl_uniform.argtypes = [P, U64, U64]
        lib.wl_exponential.argtypes = [P, U64, D, U64]
        lib.wl_substream.restype = U64
        lib.wl_substream.argtypes = [U64, U64]
        _lib = lib
    return _lib


def clike(n: int, seed: int, bcomment: bool = False, out: np.ndarray | None = None, frame: int = 0) -> np.ndarray:
    """frame > 0: records of that many lines, each opened by the separator 0x1E."""
    buf = np.empty(n, np.uint8) if out is None else out
    assert buf.dtype == np.uint8 and buf.flags.c_contiguous and buf.size == n
    _load().wl_clike(buf.ctypes.data, n, seed, 1 if bcomment else 0, int(frame))
    return buf


def json(n: int, seed: int, out: np.ndarray | None = None) -> np.ndarray:
    buf = np.empty(n, np.uint8) if out is None else out
    assert buf.dtype == np.uint8 and buf.flags.c_contiguous and buf.size == n
    _load().wl_json(buf.ctypes.data, n, seed)
    return buf


def loglines(n: int, period: int | None = 40, fill: int = ord("x")) -> np.ndarray:
    buf = np.full(n, fill, np.uint8)
    if period:
        buf[period - 1::period] = 0x0A
    return buf


def lognormal_sizes(count, median, sigma, lo, hi, seed) -> np.ndarray:
    out = np.empty(count, np.uint64)
    _load().wl_lognormal_sizes(out.ctypes.data, count, float(median), float(sigma), lo, hi, seed)
    return out


def uniform(count, seed) -> np.ndarray:
    out = np.empty(count, np.float64)
    _load().wl_uniform(out.ctypes.data, count, seed)
    return out


def exponential(count, rate, seed) -> np.ndarray:
    out = np.empty(count, np.float64)
    _load().wl_exponential(out.ctypes.data, count, float(rate), seed)
    return out


def substream(seed: int, i: int) -> int:
    return int(_load().wl_substream(seed, i))


def stray_offset(n: int, seed: int, draw: int = 0) -> int:
    """The draw-th uniformly drawn offset in [0, n) from `seed` (for the stray-byte case)."""
    u = uniform(draw + 1, seed)[draw]
    return min(int(u * n), n - 1)


# Token-set ids of the batched workload.
DOC_L, DOC_D, DOC_B = 0, 1, 2


def doc_plan(count: int, seed: int, median=16384, sigma=1.5, lo=64, hi=8 << 20):
    """Sizes and token-set ids of the batched-documents workload: sizes log-normal,
    token set C-like-L with probability .475, C-like-D .475, C-like-B .05."""
    sizes = lognormal_sizes(count, median, sigma, lo, hi, substream(seed, 0))
    u = uniform(count, substream(seed, 1))
    sets = np.where(u < 0.475, DOC_L, np.where(u < 0.95, DOC_D, DOC_B)).astype(np.uint8)
    return sizes, sets


def doc(seed: int, i: int, size: int, set_id: int) -> np.ndarray:
    """Document i of the batched workload alone (the bytes docs() places at its offset)."""
    buf = np.empty(int(size), np.uint8)
    _load().wl_clike(buf.ctypes.data, int(size), substream(seed, 1000 + i), 1 if set_id == DOC_B else 0, 0)
    return buf


def docs(count: int, seed: int, **kw):
    """Concatenated documents of the batched workload.
    Returns (bytes u8[total], offsets u64[count], sizes u64[count], set_ids u8[count])."""
    sizes, sets = doc_plan(count, seed, **kw)
    offs = np.zeros(count, np.uint64)
    if count > 1:
        offs[1:] = np.cumsum(sizes[:-1])
    total = int(sizes.sum())
    buf = np.empty(total, np.uint8)
    lib = _load()
    base = buf.ctypes.data
    for i in range(count):
        lib.wl_clike(base + int(offs[i]), int(sizes[i]), substream(seed, 1000 + i),
                     1 if sets[i] == DOC_B else 0, 0)
    return buf, offs, sizes, sets
