"""Python face of the C ABI: compile a token set once, scan device buffers many times.

Argument marshalling only -- torch tensors supply device memory and the current stream;
every step of a scan runs in liblexgpu.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import abi


def _norm_defs(defs):
    out = []
    for d in defs:
        if hasattr(d, "pattern"):
            pat, pr, dc = d.pattern, getattr(d, "priority", 0), getattr(d, "discard", False)
        elif isinstance(d, dict):
            pat, pr, dc = d["pattern"], d.get("priority", 0), d.get("discard", False)
        else:
            d = tuple(d)
            pat, pr, dc = d[0], (d[1] if len(d) > 1 else 0), (d[2] if len(d) > 2 else False)
        if isinstance(pat, str):
            pat = pat.encode("latin-1")
        out.append((pat, int(pr), bool(dc)))
    return out


def _bits_to_set(buf) -> frozenset:
    b = bytes(buf)
    return frozenset(i for i in range(256) if (b[i >> 3] >> (i & 7)) & 1)


@dataclass
class RunResult:
    kinds: "object"          # torch.uint8 [ntokens] (device)
    lens: "object"           # torch.int32 [ntokens] (device), u32 values
    offsets: "object"        # torch.int64 [ntokens] (device) or None
    ntokens: int
    error_offset: int
    status: int
    nslices: int


class Lexer:
    """A compiled token set (lex_dfa)."""

    def __init__(self, handle, ndefs: int, defs=None):
        self._h = handle
        self.ndefs = ndefs
        self.defs = defs

    # ----------------------------------------------------------------- build
    @classmethod
    def compile(cls, defs) -> "Lexer":
        return cls._compile(defs, None, False)

    @classmethod
    def compile_framed(cls, defs, reserved: int = 0x1E, reserved_discard: bool = False) -> "Lexer":
        """The set framed by a reserved byte (Section 7.1): the byte is taken out of every
        pattern and becomes kind len(defs), a token of its own."""
        return cls._compile(defs, int(reserved), reserved_discard)

    @classmethod
    def _compile(cls, defs, reserved, reserved_discard) -> "Lexer":
        L = abi.lib()
        nd = _norm_defs(defs)
        arr = (abi.TokDef * len(nd))()
        keep = []
        for i, (p, pr, dc) in enumerate(nd):
            keep.append(p)
            arr[i].pattern = p
            arr[i].priority = pr
            arr[i].discard = 1 if dc else 0
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        if reserved is None:
            rc = L.lex_compile(arr, len(nd), C.byref(h), err, 512)
        else:
            rc = L.lex_compile_framed(arr, len(nd), reserved, 1 if reserved_discard else 0, C.byref(h), err, 512)
        abi.check(rc, err.value.decode("latin-1"))
        if reserved is not None:
            nd = list(nd) + [(("\\x%02X" % reserved).encode(), 0, bool(reserved_discard))]
        return cls(h, len(nd), nd)

    @classmethod
    def from_table(cls, next_table, accept, q0: int = 0, discard=None) -> "Lexer":
        L = abi.lib()
        nxt = np.ascontiguousarray(np.asarray(next_table, dtype=np.int32))
        acc = np.ascontiguousarray(np.asarray(accept, dtype=np.int32))
        n = acc.size
        assert nxt.shape == (n, 256)
        ntok = int(acc.max()) + 1 if n and acc.max() >= 0 else 0
        disc = np.zeros(max(ntok, 1), np.uint8)
        if discard is not None:
            d = np.asarray(discard, np.uint8)
            ntok = max(ntok, d.size)
            disc = np.zeros(max(ntok, 1), np.uint8)
            disc[: d.size] = d
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        rc = L.lex_compile_table(n, q0, nxt.ctypes.data, acc.ctypes.data, disc.ctypes.data, ntok,
                                 C.byref(h), err, 512)
        abi.check(rc, err.value.decode("latin-1"))
        return cls(h, ntok)

    def close(self):
        if getattr(self, "_h", None) and abi._lib is not None:
            abi._lib.lex_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- queries
    def cert(self, mode: int = abi.LEX_MODE_EXACT, raw: bool = False) -> frozenset:
        buf = (C.c_uint8 * 32)()
        abi.check(abi.lib().lex_cert(self._h, mode, 1 if raw else 0, buf))
        return _bits_to_set(buf)

    def info(self) -> dict:
        i = abi.Info()
        abi.check(abi.lib().lex_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in abi.Info._fields_ if k != "reserved"}

    def tables(self, mode: int):
        nrows = self.info()["nrows"]
        t = np.empty(nrows * 256, np.uint32)
        ri = np.empty(nrows, np.uint8)
        rk = np.empty(nrows, np.uint8)
        abi.check(abi.lib().lex_tables(self._h, mode, t.ctypes.data, t.size, ri.ctypes.data, rk.ctypes.data,
                                       nrows))
        return t, ri, rk

    def plan(self, n: int, mode: int = abi.LEX_MODE_EXACT, opts: abi.RunOpts | None = None) -> dict:
        """The configuration a scan of n bytes would use: lane_bytes, block_threads, path
        (1 pipeline, 2 fused, 3 one pass) and windowed."""
        out = abi.PlanInfo()
        abi.check(abi.lib().lex_plan(self._h, n, mode, C.byref(opts) if opts else None, C.byref(out)), "lex_plan")
        return {k: getattr(out, k) for k, _ in abi.PlanInfo._fields_}

    def workspace_size(self, n: int, mode: int, opts: abi.RunOpts | None = None) -> int:
        ws = abi.lib().lex_workspace_size(self._h, n, mode, C.byref(opts) if opts else None)
        if ws == 0:
            raise abi.LexError(abi.LEX_EINVAL, "no workspace size for these arguments")
        return ws

    # ---------------------------------------------------------------- scans
    def run_into(self, data, n: int, mode: int, kinds, lens, offsets, cap: int, result, ws,
                 opts: abi.RunOpts | None = None, stream=None):
        """Enqueues one scan into caller-owned device tensors (no allocation, no sync)."""
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        rc = abi.lib().lex_run(self._h, data.data_ptr() if n else None, n, mode,
                               kinds.data_ptr() if cap else None, lens.data_ptr() if cap else None,
                               offsets.data_ptr() if offsets is not None else None, cap,
                               result.data_ptr(), ws.data_ptr(), ws.numel(),
                               C.byref(opts) if opts else None, C.c_void_p(s.cuda_stream))
        abi.check(rc, "lex_run")

    def run_static_into(self, data, n: int, mode: int, kinds, lens, offsets, cap: int, result,
                        opts: abi.RunOpts | None = None, stream=None):
        """As run_into, with the library's own scratch as workspace (lex_run_static): for
        callers that cannot allocate.  Scans that overlap on one device race."""
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        rc = abi.lib().lex_run_static(self._h, data.data_ptr() if n else None, n, mode,
                                      kinds.data_ptr() if cap else None, lens.data_ptr() if cap else None,
                                      offsets.data_ptr() if offsets is not None else None, cap,
                                      result.data_ptr(), C.byref(opts) if opts else None,
                                      C.c_void_p(s.cuda_stream))
        abi.check(rc, "lex_run_static")

    def run(self, data, mode: int = abi.LEX_MODE_EXACT, offsets: bool = False, cap: int | None = None,
            opts: abi.RunOpts | None = None) -> RunResult:
        """Scans a 1-D uint8 CUDA tensor; synchronises once to read the result."""
        import torch

        if not (data.is_cuda and data.dtype == torch.uint8 and data.dim() == 1 and data.is_contiguous()):
            raise abi.LexError(abi.LEX_EINVAL, "data must be a contiguous 1-D uint8 CUDA tensor")
        n = data.numel()
        dev = data.device
        cap = n if cap is None else cap
        kinds = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        lens = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        offs = torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if offsets else None
        res = torch.zeros(3, dtype=torch.int64, device=dev)
        ws = torch.empty(self.workspace_size(n, mode, opts), dtype=torch.uint8, device=dev)
        self.run_into(data, n, mode, kinds, lens, offs, cap, res, ws, opts)
        r = res.cpu().numpy()
        ntok, err = int(r[0]), int(r[1])
        status = int(np.int32(r[2] & 0xFFFFFFFF))
        nsl = int((int(r[2]) >> 32) & 0xFFFFFFFF)
        k = min(ntok, cap) if status == 0 else 0
        return RunResult(kinds[:k], lens[:k], offs[:k] if offs is not None else None, ntok, err, status, nsl)

    def cpu_chunked(self, data, mode: int = abi.LEX_MODE_EXACT, chunk_bytes: int = 64 << 10, threads: int = 0,
                    kinds=None, lens=None):
        """The host baseline (lex_cpu_chunked): the paper's multithreaded chunked executor
        on the CPU cores over this lexer's tables.  data: a uint8 numpy array; kinds/lens:
        optional preallocated numpy outputs of at least data.size entries.  Returns
        (kinds, lens, ntokens, error_offset, nchunks); kinds/lens are views of length
        ntokens.  Not a GPU path."""
        w = np.ascontiguousarray(data, dtype=np.uint8)
        n = w.size
        if kinds is None:
            kinds = np.empty(max(n, 1), np.uint8)
        if lens is None:
            lens = np.empty(max(n, 1), np.uint32)
        assert kinds.dtype == np.uint8 and lens.dtype == np.uint32
        r = abi.Result()
        abi.check(abi.lib().lex_cpu_chunked(self._h, w.ctypes.data if n else None, n, mode, kinds.ctypes.data,
                                            lens.ctypes.data, min(kinds.size, lens.size) if n else 0,
                                            chunk_bytes, threads, C.byref(r)), "lex_cpu_chunked")
        k = r.ntokens
        return kinds[:k], lens[:k], k, r.error_offset, r.nslices

    def cert_bitmap(self, data, mode: int = abi.LEX_MODE_EXACT):
        import torch

        n = data.numel()
        bits = torch.zeros(max((n + 63) // 64, 1), dtype=torch.int64, device=data.device)
        s = torch.cuda.current_stream()
        abi.check(abi.lib().lex_cert_bitmap(self._h, data.data_ptr() if n else None, n, mode,
                                            bits.data_ptr(), C.c_void_p(s.cuda_stream)))
        return bits


@dataclass
class BatchResult:
    kinds: "object"       # torch.uint8 [ntokens] (device)
    lens: "object"        # torch.int32 [ntokens] (device), u32 values
    offsets: "object"     # torch.int64 [ntokens] (device, relative to each document) or None
    docs: "object"        # numpy structured array: tok_offset, ntokens, error_offset, status, nslices
    ntokens: int
    nerrors: int          # documents that did not tokenize completely
    status: int
    nslices: int


DOC_DTYPE = np.dtype([("offset", "<u8"), ("length", "<u4"), ("inst", "<u2"), ("flags", "<u2")])
DOC_RESULT_DTYPE = np.dtype([("tok_offset", "<u8"), ("ntokens", "<u8"), ("error_offset", "<u8"),
                             ("status", "<i4"), ("nslices", "<u4")])


class Batch:
    """Several (lexer, mode) instances resident together for batched document scans
    (lex_batch).  Documents are described by DOC_DTYPE records."""

    def __init__(self, instances):
        """instances: [(Lexer, mode), ...] (at most 8)."""
        L = abi.lib()
        self._keep = [lx for lx, _ in instances]
        hs = (C.c_void_p * len(instances))(*[lx._h for lx, _ in instances])
        ms = (C.c_int32 * len(instances))(*[int(m) for _, m in instances])
        out = C.c_void_p()
        err = C.create_string_buffer(512)
        abi.check(L.lex_batch_create(hs, ms, len(instances), C.byref(out), err, 512), err.value.decode())
        self._h = out.value

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            try:
                abi.lib().lex_batch_free(h)
            except Exception:
                pass

    def workspace_size(self, ndocs: int, nbytes: int, opts: abi.RunOpts | None = None) -> int:
        return abi.lib().lex_batch_workspace_size(self._h, ndocs, nbytes, C.byref(opts) if opts else None)

    def run_into(self, data, nbytes, docs_dev, ndocs, kinds, lens, offsets, cap, res_dev, total_dev, ws,
                 opts: abi.RunOpts | None = None, stream=None):
        """Enqueues one batched scan on `stream` (torch stream; default: current); device
        tensors throughout.  Capturable in a CUDA graph."""
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        abi.check(abi.lib().lex_run_batch(
            self._h, data.data_ptr() if nbytes else None, nbytes, docs_dev.data_ptr() if ndocs else None,
            ndocs, kinds.data_ptr(), lens.data_ptr(), offsets.data_ptr() if offsets is not None else None,
            cap, res_dev.data_ptr() if ndocs else None, total_dev.data_ptr(), ws.data_ptr(), ws.numel(),
            C.byref(opts) if opts else None, C.c_void_p(s.cuda_stream)))

    def run(self, data, docs: np.ndarray, offsets: bool = False, cap: int | None = None,
            opts: abi.RunOpts | None = None) -> BatchResult:
        """Scans the documents `docs` (DOC_DTYPE records) of the uint8 CUDA tensor `data`."""
        import torch

        dev = data.device
        n = data.numel()
        docs = np.ascontiguousarray(docs, dtype=DOC_DTYPE)
        nd = docs.size
        cap = n if cap is None else cap
        docs_dev = torch.from_numpy(docs.view(np.uint8).copy()).to(dev)
        kinds = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        lens = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        offs = torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if offsets else None
        res = torch.empty(max(nd, 1) * 32, dtype=torch.uint8, device=dev)
        total = torch.zeros(3, dtype=torch.int64, device=dev)
        ws = torch.empty(self.workspace_size(nd, n, opts), dtype=torch.uint8, device=dev)
        self.run_into(data, n, docs_dev, nd, kinds, lens, offs, cap, res, total, ws, opts)
        t = total.cpu().numpy()
        per = res.cpu().numpy()[: nd * 32].view(DOC_RESULT_DTYPE)
        ntok, nerr = int(t[0]), int(t[1])
        status = int(np.int32(t[2] & 0xFFFFFFFF))
        nsl = int((int(t[2]) >> 32) & 0xFFFFFFFF)
        k = min(ntok, cap) if status == 0 else 0
        return BatchResult(kinds[:k], lens[:k], offs[:k] if offs is not None else None, per, ntok, nerr,
                           status, nsl)
