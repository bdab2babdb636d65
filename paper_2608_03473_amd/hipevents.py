"""Raw hipEvent_t handles through ctypes (plumbing for per-phase timing of a scan).

torch.cuda.Event only sees torch's own stream operations lazily; the scan records its
phase boundaries itself (lex_run_opts.events), so the caller needs plain HIP events.
"""
from __future__ import annotations

import ctypes as C

_hip = None


def _lib():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise OSError("libamdhip64 not found")
        _hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        _hip.hipEventDestroy.argtypes = [C.c_void_p]
        _hip.hipEventSynchronize.argtypes = [C.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        _hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
    return _hip


class PhaseEvents:
    """LEX_NPHASES + 1 events for lex_run_opts.events, and their elapsed times."""

    def __init__(self, n: int = 5):
        L = _lib()
        self.ev = (C.c_void_p * n)()
        for i in range(n):
            h = C.c_void_p()
            rc = L.hipEventCreate(C.byref(h))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed: {rc}")
            self.ev[i] = h
        self.n = n

    @property
    def array(self):
        return C.cast(self.ev, C.c_void_p)

    def elapsed_ms(self):
        """Milliseconds of each phase: [i] = event i -> event i+1."""
        L = _lib()
        L.hipEventSynchronize(self.ev[self.n - 1])
        out = []
        for i in range(self.n - 1):
            f = C.c_float()
            rc = L.hipEventElapsedTime(C.byref(f), self.ev[i], self.ev[i + 1])
            if rc != 0:
                raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
            out.append(f.value)
        return out

    def close(self):
        if self.ev is not None:
            L = _lib()
            for i in range(self.n):
                L.hipEventDestroy(self.ev[i])
            self.ev = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StreamTimer:
    """Times work enqueued on a HIP stream (passed as its handle) between two events."""

    def __init__(self):
        self.ev = PhaseEvents(2)

    def __enter__(self):
        return self

    def start(self, stream_handle):
        _lib().hipEventRecord(self.ev.ev[0], C.c_void_p(stream_handle))

    def stop(self, stream_handle) -> None:
        _lib().hipEventRecord(self.ev.ev[1], C.c_void_p(stream_handle))

    def ms(self) -> float:
        return self.ev.elapsed_ms()[0]

    def __exit__(self, *exc):
        self.ev.close()
