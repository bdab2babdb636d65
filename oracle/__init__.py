"""Reference (oracle) implementation of certified-split lexing -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product library never does, and this package never imports the
product: the two share no code.  The native part (``oracle.cc``) is a plain serial C++
implementation; this module only marshals arguments through ctypes.

What it computes (see oracle.cc for the paper map):
  * ``OracleSet.lex``         -- the serial longest-match scan of Section 3, matching each
                                 token definition directly with its own Thompson NFA;
  * ``OracleSet.cert``        -- Definitions 1-3 and the useful sets (Corollary 2,
                                 Proposition 2) on an automaton the oracle builds itself;
  * ``OracleSet.witness``     -- the witness of Theorem 2;
  * ``OracleSet.lex_chunked`` -- the chunked scan of Theorems 1 and 3 with Corollary 1's
                                 truncation;
  * ``OracleSet.bruteforce``  -- the exhaustive sweep of Section 6.1 plus the lemma checks;
  * ``cert_table``            -- certificates of a hand-built automaton (Section 4.1);
  * ``OracleSet(defs, reserved=r)`` -- the set framed by a reserved byte (Section 7.1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A mutation test points this at a deliberately broken build of oracle.cc.
_LIB_LOAD = os.environ.get("ORACLE_LIB_OVERRIDE", _LIB_PATH)

BF_FIELDS = (
    "strings", "tokenizable", "lemma1_viol", "thm1_viol", "cor1_viol", "thm3_viol",
    "malformed_i_viol", "prop3_viol", "witness_viol", "necessity_found", "necessity_viol",
    "pairs_consumed", "pairs_admitted_i", "pairs_refused_safe", "mode_splits",
)


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with the host compiler (plain g++ -O2)."""
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Wextra",
           "-o", _LIB_PATH, os.path.join(_HERE, "oracle.cc")]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Def(C.Structure):
    _fields_ = [("pattern", C.c_char_p), ("priority", C.c_int32), ("discard", C.c_uint8)]


class _CertInfo(C.Structure):
    _fields_ = [("exact_raw", C.c_uint8 * 32), ("discard_raw", C.c_uint8 * 32),
                ("exact_useful", C.c_uint8 * 32), ("discard_useful", C.c_uint8 * 32),
                ("q0_live", C.c_uint8 * 32), ("consumed", C.c_uint8 * 32),
                ("nstates", C.c_int32), ("q0_live_state", C.c_int32),
                ("reentrant", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_LOAD == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_LOAD)
    P = C.c_void_p
    lib.orc_compile.restype = P
    lib.orc_compile.argtypes = [P, C.c_uint32, C.c_char_p, C.c_size_t]
    lib.orc_compile_framed.restype = P
    lib.orc_compile_framed.argtypes = [P, C.c_uint32, C.c_uint32, C.c_int, C.c_char_p, C.c_size_t]
    lib.orc_free.argtypes = [P]
    lib.orc_nkinds.restype = C.c_uint32
    lib.orc_nkinds.argtypes = [P]
    lib.orc_lex.argtypes = [P, P, C.c_uint64, C.c_int, P, P, P, C.c_uint64,
                            C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.orc_cert.argtypes = [P, C.POINTER(_CertInfo)]
    lib.orc_cert_table.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.POINTER(_CertInfo)]
    lib.orc_witness.restype = C.c_int64
    lib.orc_witness.argtypes = [P, C.c_int, P, C.c_uint64, C.POINTER(C.c_uint64)]
    lib.orc_lex_chunked.argtypes = [P, P, C.c_uint64, P, C.c_uint64, C.c_int, P, P, C.c_uint64,
                                    C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.orc_bruteforce.argtypes = [P, P, C.c_uint32, C.c_uint32, P]
    _lib = lib
    return lib


def _bits(arr) -> frozenset:
    b = bytes(arr)
    return frozenset(i for i in range(256) if (b[i >> 3] >> (i & 7)) & 1)


def _info_dict(info: _CertInfo) -> dict:
    return {
        "exact_raw": _bits(info.exact_raw), "discard_raw": _bits(info.discard_raw),
        "exact": _bits(info.exact_useful), "discard": _bits(info.discard_useful),
        "q0_live": _bits(info.q0_live), "consumed": _bits(info.consumed),
        "nstates": info.nstates, "q0_live_state": bool(info.q0_live_state),
        "reentrant": bool(info.reentrant),
    }


def _as_u8(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    a = np.ascontiguousarray(data, dtype=np.uint8)
    return a


def _norm_defs(defs):
    """Accepts dicts {pattern, priority, discard} or tuples (pattern[, priority[, discard]])."""
    out = []
    for d in defs:
        if isinstance(d, dict):
            pat, pr, dc = d["pattern"], d.get("priority", 0), d.get("discard", False)
        else:
            d = tuple(d)
            pat = d[0]
            pr = d[1] if len(d) > 1 else 0
            dc = d[2] if len(d) > 2 else False
        if isinstance(pat, str):
            pat = pat.encode("latin-1")
        out.append((pat, int(pr), bool(dc)))
    return out


class OracleSet:
    """A token set compiled by the oracle (patterns -> per-kind Thompson NFAs)."""

    def __init__(self, defs, reserved: int | None = None, reserved_discard: bool = False):
        """reserved: frame the set by that byte (Section 7.1): it leaves every pattern and
        becomes kind len(defs), a one-byte token of its own."""
        lib = _load()
        self.defs = _norm_defs(defs)
        arr = (_Def * len(self.defs))()
        self._keep = []
        for i, (p, pr, dc) in enumerate(self.defs):
            self._keep.append(p)
            arr[i].pattern = p
            arr[i].priority = pr
            arr[i].discard = 1 if dc else 0
        err = C.create_string_buffer(256)
        if reserved is None:
            h = lib.orc_compile(arr, len(self.defs), err, 256)
        else:
            h = lib.orc_compile_framed(arr, len(self.defs), int(reserved), 1 if reserved_discard else 0, err, 256)
        if not h:
            raise ValueError(err.value.decode("latin-1"))
        self._h = h
        self.nkinds = lib.orc_nkinds(h)
        if reserved is not None:
            self.defs = self.defs + [(b"(reserved byte)", 0, bool(reserved_discard))]
        self.discard_kinds = frozenset(i for i, d in enumerate(self.defs) if d[2])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def lex(self, data, discard: bool = False, offsets: bool = False):
        """Serial scan.  Returns (kinds u8, lens u32, con) or with offsets (kinds, lens, offs, con)."""
        w = _as_u8(data)
        n = w.size
        cap = n
        kinds = np.empty(max(cap, 1), np.uint8)
        lens = np.empty(max(cap, 1), np.uint32)
        offs = np.empty(max(cap, 1), np.uint64) if offsets else None
        ntok, con = C.c_uint64(), C.c_uint64()
        rc = _lib.orc_lex(self._h, w.ctypes.data, n, 1 if discard else 0, kinds.ctypes.data,
                          lens.ctypes.data, offs.ctypes.data if offsets else None, cap,
                          C.byref(ntok), C.byref(con))
        if rc != 0:
            raise RuntimeError(f"orc_lex failed: {rc}")
        k = ntok.value
        if offsets:
            return kinds[:k].copy(), lens[:k].copy(), offs[:k].copy(), con.value
        return kinds[:k].copy(), lens[:k].copy(), con.value

    def cert(self) -> dict:
        info = _CertInfo()
        rc = _lib.orc_cert(self._h, C.byref(info))
        if rc != 0:
            raise RuntimeError(f"orc_cert failed: {rc}")
        return _info_dict(info)

    def witness(self, b: int):
        buf = np.empty(4096, np.uint8)
        boff = C.c_uint64()
        r = _lib.orc_witness(self._h, int(b), buf.ctypes.data, buf.size, C.byref(boff))
        if r < 0:
            raise RuntimeError(f"orc_witness failed: {r}")
        if r == 0:
            return None
        return bytes(buf[:r]), boff.value

    def lex_chunked(self, data, cuts, discard: bool = False):
        w = _as_u8(data)
        c = np.ascontiguousarray(np.asarray(cuts, dtype=np.uint64))
        cap = max(w.size, 1)
        kinds = np.empty(cap, np.uint8)
        lens = np.empty(cap, np.uint32)
        ntok, err = C.c_uint64(), C.c_uint64()
        rc = _lib.orc_lex_chunked(self._h, w.ctypes.data, w.size, c.ctypes.data if c.size else None,
                                  c.size, 1 if discard else 0, kinds.ctypes.data, lens.ctypes.data,
                                  cap, C.byref(ntok), C.byref(err))
        if rc != 0:
            raise RuntimeError(f"orc_lex_chunked failed: {rc}")
        k = ntok.value
        return kinds[:k].copy(), lens[:k].copy(), err.value

    def bruteforce(self, alphabet: bytes, maxlen: int) -> dict:
        a = np.frombuffer(bytes(alphabet), np.uint8)
        st = np.zeros(len(BF_FIELDS), np.uint64)
        rc = _lib.orc_bruteforce(self._h, a.ctypes.data, a.size, maxlen, st.ctypes.data)
        if rc != 0:
            raise RuntimeError(f"orc_bruteforce failed: {rc}")
        return {k: int(v) for k, v in zip(BF_FIELDS, st)}


def cert_table(next_table, accept, q0: int = 0, discard=None) -> dict:
    """Certificates of a hand-built automaton.  next_table: (n, 256) ints, -1 = undefined;
    accept: n ints, -1 = not accepting, else a token index; discard: per-token flags."""
    lib = _load()
    nxt = np.ascontiguousarray(np.asarray(next_table, dtype=np.int32))
    acc = np.ascontiguousarray(np.asarray(accept, dtype=np.int32))
    n = acc.size
    assert nxt.shape == (n, 256)
    ntok = int(acc.max()) + 1 if n and acc.max() >= 0 else 0
    if discard is None:
        discard = [0] * max(ntok, 1)
    disc = np.ascontiguousarray(np.asarray(discard, dtype=np.uint8))
    ntok = max(ntok, disc.size)
    info = _CertInfo()
    rc = lib.orc_cert_table(n, q0, nxt.ctypes.data, acc.ctypes.data, disc.ctypes.data, ntok,
                            C.byref(info))
    if rc != 0:
        raise RuntimeError(f"orc_cert_table failed: {rc}")
    return _info_dict(info)
