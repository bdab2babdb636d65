"""The C-ABI library loads and exports every function include/lex.h declares; argument
checking that happens on the host.  CPU only: no scan is launched."""
import ctypes as C
import os
import re

import numpy as np

import pytest

import paper_2608_03473_amd as P
from workloads import tokensets as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(lex_\w+)\s*\(", src, flags=re.M))
    return names


def test_every_declared_symbol_is_exported():
    names = declared()
    assert {"lex_compile", "lex_run", "lex_free", "lex_cert"} <= names
    lib = C.CDLL(P.lib_path())
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} declared but not exported"


def test_host_side_argument_checks():
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    L = P.lib()
    assert L.lex_workspace_size(lx._h, 1 << 20, 7, None) == 0  # bad mode
    bad = P.RunOpts(lane_bytes=24)  # not a multiple of 16
    assert L.lex_workspace_size(lx._h, 1 << 20, 0, C.byref(bad)) == 0
    bad = P.RunOpts(lane_bytes=1024, chunk_bytes=1000)  # lanes must divide chunks
    assert L.lex_workspace_size(lx._h, 1 << 20, 0, C.byref(bad)) == 0
    assert L.lex_workspace_size(lx._h, 1 << 33, 0, None) == 0  # beyond 32-bit offsets
    bad = P.RunOpts(emit=5)  # unknown emit choice
    assert L.lex_workspace_size(lx._h, 1 << 20, 0, C.byref(bad)) == 0
    # the windowed emit keeps checkpoints: a larger workspace than the lane emit
    lane = P.RunOpts(emit=P.LEX_EMIT_LANE)
    assert lx.workspace_size(1 << 20, 0) > L.lex_workspace_size(lx._h, 1 << 20, 0, C.byref(lane)) > 0
    rc = L.lex_run(lx._h, None, 10, 0, None, None, None, 0, None, None, 0, None, None)
    assert rc == P.LEX_EINVAL
    assert lx.workspace_size(1 << 20, 0) > 0


def test_framed_compile_checks():
    """lex_compile_framed (Section 7.1): argument checks, the reserved byte's kind, and the
    certified plan of a framed C-like-B set (no hybrid plan)."""
    L = P.lib()
    defs = T.as_tuples(T.CLIKE_B)
    arr = (P.abi.TokDef * len(defs))()
    keep = [p.encode() for p, _, _ in defs]
    for i, (p, pr, dc) in enumerate(defs):
        arr[i].pattern, arr[i].priority, arr[i].discard = keep[i], pr, int(dc)
    h = C.c_void_p()
    assert L.lex_compile_framed(arr, len(defs), 256, 0, C.byref(h), None, 0) == P.LEX_EINVAL
    assert L.lex_compile_framed(None, 1, 0x1E, 0, C.byref(h), None, 0) == P.LEX_EINVAL
    many = (P.abi.TokDef * 255)()
    for i in range(255):
        many[i].pattern = b"a"
    assert L.lex_compile_framed(many, 255, 0x1E, 0, C.byref(h), None, 0) == P.LEX_ELIMIT
    lx = P.Lexer.compile_framed(defs)
    assert lx.info()["nkinds"] == len(defs) + 1
    for mode in (P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD):
        assert lx.cert(mode) == {0x1E}
        assert lx.plan(64 << 20, mode)["hybrid"] == 0
        assert P.Lexer.compile(defs).plan(64 << 20, mode)["hybrid"] == 1
    # a rule that was the reserved byte alone keeps a valid, empty language
    lx = P.Lexer.compile_framed([(r"\x1E", 0, False), (r"[a-z]+", 0, False)])
    assert lx.cert() == {0x1E}


def test_plan_query():
    """lex_plan reports what lex_run would use: one pass by default where the windowed emit
    applies (256-lane workgroups), the fused path otherwise, the pipeline when asked."""
    cl = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    js = P.Lexer.compile(T.as_tuples(T.JSON))
    d = cl.plan(512 << 20)
    assert d == {"lane_bytes": 2048, "block_threads": 256, "path": 3, "windowed": 1, "hybrid": 0}
    cb = P.Lexer.compile(T.as_tuples(T.CLIKE_B))  # refused: the hybrid plan above one speculative lane
    h = cb.plan(1 << 20, P.LEX_MODE_DISCARD)
    assert h["hybrid"] == 1 and h["path"] == 1 and h["lane_bytes"] == 4096
    assert cb.plan(1 << 20, P.LEX_MODE_DISCARD, P.RunOpts(lane_bytes=8192))["lane_bytes"] == 8192
    assert cb.plan(4096, P.LEX_MODE_DISCARD)["hybrid"] == 0
    assert cb.plan(1 << 20, P.LEX_MODE_DISCARD | P.LEX_MODE_SERIAL)["hybrid"] == 0
    assert cl.plan(512 << 20, opts=P.RunOpts(path=2))["lane_bytes"] == 1024
    assert cl.plan(512 << 20, opts=P.RunOpts(path=2))["path"] == 2
    assert cl.plan(512 << 20, opts=P.RunOpts(path=1))["path"] == 1
    assert cl.plan(512 << 20, opts=P.RunOpts(emit=P.LEX_EMIT_LANE)) ["path"] == 2
    assert cl.plan(512 << 20, opts=P.RunOpts(block_threads=1024))["path"] == 2  # default path, other block
    j = js.plan(256 << 20, P.LEX_MODE_DISCARD)  # not monotone: windowed emit, no one pass
    assert j["path"] == 2 and j["windowed"] == 1
    cd = P.Lexer.compile(T.as_tuples(T.CLIKE_D))  # discarded kinds, monotone: one pass
    assert cd.plan(512 << 20, P.LEX_MODE_DISCARD)["path"] == 3
    assert cd.plan(512 << 20, P.LEX_MODE_DISCARD)["windowed"] == 1
    assert js.plan(256 << 20, P.LEX_MODE_DISCARD, P.RunOpts(path=3))["path"] == 2
    with pytest.raises(P.LexError):
        cl.plan(1 << 20, opts=P.RunOpts(path=3, block_threads=1024))  # one pass uses 256
    with pytest.raises(P.LexError):
        cl.plan(1 << 20, opts=P.RunOpts(path=4))
    with pytest.raises(P.LexError):
        cl.plan(1 << 33)


def test_info_and_tables():
    lx = P.Lexer.compile(T.as_tuples(T.JSON))
    info = lx.info()
    assert info["monotone"] == 0 and info["nrows"] == info["nstates"] + 3
    t, ri, rk = lx.tables(1)
    assert t.size == info["nrows"] * 256 and ri.size == info["nrows"]
    # every next-row field points at a row of the table
    assert int(((t & 0x00FFFC00) >> 10).max()) < info["nrows"]
    # the swizzle field matches the next row
    assert np.array_equal((t >> 2) & 31, ((t >> 10) & 0x3FFF) & 31)


def test_batch_argument_checks():
    """lex_batch_create validates on the host before touching a device."""
    L = P.lib()
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    out = C.c_void_p()
    err = C.create_string_buffer(256)
    hs = (C.c_void_p * 9)(*([lx._h] * 9))
    ms = (C.c_int32 * 9)(*([0] * 9))
    assert L.lex_batch_create(None, ms, 1, C.byref(out), err, 256) == P.LEX_EINVAL
    assert L.lex_batch_create(hs, ms, 0, C.byref(out), err, 256) == P.LEX_EINVAL
    assert L.lex_batch_create(hs, ms, 9, C.byref(out), err, 256) == P.LEX_ELIMIT
    bad = (C.c_int32 * 1)(2)  # serial is a per-document flag, not an instance mode
    assert L.lex_batch_create(hs, bad, 1, C.byref(out), err, 256) == P.LEX_EINVAL
    assert L.lex_batch_workspace_size(None, 10, 1000, None) == 0
    assert L.lex_run_batch(None, None, 0, None, 0, None, None, None, 0, None, None, None, 0, None, None) == P.LEX_EINVAL
    assert np.dtype(P.DOC_DTYPE).itemsize == 16 and np.dtype(P.DOC_RESULT_DTYPE).itemsize == 32


def test_size_limit_boundary():
    """Offsets are 32-bit: n = 2^32 - 16 is the largest input; one byte more is LEX_ELIMIT from
    the host checks of lex_workspace_size, lex_plan and lex_run (no device work happens; the
    pointers below are never dereferenced)."""
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    L = P.lib()
    top = (1 << 32) - 16
    assert L.lex_workspace_size(lx._h, top, 0, None) > 0
    assert lx.plan(top, 0)["path"] in (1, 2, 3)
    assert L.lex_workspace_size(lx._h, top + 1, 0, None) == 0
    info = P.abi.PlanInfo()
    assert L.lex_plan(lx._h, top + 1, 0, None, C.byref(info)) == P.LEX_ELIMIT
    fake = C.c_void_p(1 << 20)  # 16-byte aligned, never touched
    rc = L.lex_run(lx._h, fake, top + 1, 0, fake, fake, None, 0, fake, fake, 1 << 20, None, None)
    assert rc == P.LEX_ELIMIT
