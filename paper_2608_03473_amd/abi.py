"""ctypes declarations of include/lex.h (names and layouts mirror the header)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(HERE, "liblexgpu.so")

LEX_OK, LEX_EINVAL, LEX_ESYNTAX, LEX_ENOMEM, LEX_EOVERFLOW, LEX_EDEVICE, LEX_ELIMIT = 0, -1, -2, -3, -4, -5, -6
LEX_MODE_EXACT, LEX_MODE_DISCARD, LEX_MODE_SERIAL = 0, 1, 2
_NAMES = {LEX_EINVAL: "LEX_EINVAL", LEX_ESYNTAX: "LEX_ESYNTAX", LEX_ENOMEM: "LEX_ENOMEM",
          LEX_EOVERFLOW: "LEX_EOVERFLOW", LEX_EDEVICE: "LEX_EDEVICE", LEX_ELIMIT: "LEX_ELIMIT"}


class LexError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}" if msg else _NAMES.get(code, str(code)))
        self.code = code


class TokDef(C.Structure):
    _fields_ = [("pattern", C.c_char_p), ("priority", C.c_int32), ("discard", C.c_uint8)]


class Result(C.Structure):
    _fields_ = [("ntokens", C.c_uint64), ("error_offset", C.c_uint64), ("status", C.c_int32),
                ("nslices", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("nkinds", C.c_int32), ("nstates", C.c_int32), ("nclasses", C.c_int32),
                ("nrows", C.c_int32), ("reentrant", C.c_int32), ("monotone", C.c_int32),
                ("q0_live", C.c_int32), ("reserved", C.c_int32)]


LEX_NPHASES = 4
LEX_STATIC_WS_BYTES = 64 << 20  # scratch of lex_run_static per device
LEX_EMIT_DEFAULT, LEX_EMIT_LANE = 0, 1


class PlanInfo(C.Structure):
    _fields_ = [("lane_bytes", C.c_uint32), ("block_threads", C.c_uint32), ("path", C.c_int32),
                ("windowed", C.c_int32), ("hybrid", C.c_int32)]


class RunOpts(C.Structure):
    _fields_ = [("chunk_bytes", C.c_uint64), ("lane_bytes", C.c_uint32), ("path", C.c_int32),
                ("block_threads", C.c_int32), ("emit", C.c_int32), ("events", C.c_void_p)]


_lib = None


def lib_path() -> str:
    return _LIB


def lib():
    """Loads liblexgpu.so (building it in-tree if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        from . import build
        build.build()
    L = C.CDLL(_LIB)
    P, U8, I32, U32, U64, SZ = C.c_void_p, C.c_uint8, C.c_int32, C.c_uint32, C.c_uint64, C.c_size_t
    sig = {
        "lex_compile": (C.c_int, [P, U32, P, C.c_char_p, SZ]),
        "lex_compile_framed": (C.c_int, [P, U32, U32, C.c_int, P, C.c_char_p, SZ]),
        "lex_compile_table": (C.c_int, [I32, I32, P, P, P, I32, P, C.c_char_p, SZ]),
        "lex_free": (None, [P]),
        "lex_cert": (C.c_int, [P, C.c_int, C.c_int, P]),
        "lex_info": (C.c_int, [P, C.POINTER(Info)]),
        "lex_tables": (C.c_int, [P, C.c_int, P, SZ, P, P, SZ]),
        "lex_workspace_size": (SZ, [P, U64, C.c_int, P]),
        "lex_plan": (C.c_int, [P, U64, C.c_int, P, P]),
        "lex_run": (C.c_int, [P, P, U64, C.c_int, P, P, P, U64, P, P, SZ, P, P]),
        "lex_run_static": (C.c_int, [P, P, U64, C.c_int, P, P, P, U64, P, P, P]),
        "lex_cpu_chunked": (C.c_int, [P, P, U64, C.c_int, P, P, U64, U64, U32, C.POINTER(Result)]),
        "lex_cert_bitmap": (C.c_int, [P, P, U64, C.c_int, P, P]),
        "lex_batch_create": (C.c_int, [P, P, U32, P, C.c_char_p, SZ]),
        "lex_batch_free": (None, [P]),
        "lex_batch_workspace_size": (SZ, [P, U32, U64, P]),
        "lex_run_batch": (C.c_int, [P, P, U64, P, U32, P, P, P, U64, P, P, P, SZ, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int, msg: str = ""):
    if rc != LEX_OK:
        raise LexError(rc, msg)
    return rc


def exported_symbols():
    return sorted(n for n in ("lex_compile", "lex_compile_framed", "lex_compile_table", "lex_free", "lex_cert", "lex_info",
                              "lex_tables", "lex_workspace_size", "lex_plan", "lex_run", "lex_run_static", "lex_cpu_chunked",
                              "lex_cert_bitmap",
                              "lex_batch_create", "lex_batch_free", "lex_batch_workspace_size",
                              "lex_run_batch"))
