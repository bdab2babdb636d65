"""Serving loop: lex requests under open-loop arrivals, continuously batched onto the GPU.

Every request is one document (bytes + one of the resident (lexer, mode) instances); its
result is that document's scan, bit for bit the same whether it runs alone or batched with
others (each document of a batch is scanned independently: lex_run_batch).

The server keeps the lexers' tables resident (one lex_batch) and runs K slots.  A slot
owns a stream (default priority), preallocated device buffers (input, kinds, lengths,
document table, results, workspace) and pinned host staging.  Admission is against the HBM
budget: every slot's device memory -- 6 bytes per input byte of its capacity (input and
worst-case output, since a scan has at most one token per byte), 48 bytes per document
record and result, and the batch workspace for that capacity -- counts against it, and
the slot capacity is the largest (up to slot_cap) for which the K slots fit.  A request
larger than a slot, or one arriving while the queue of admitted requests waiting for a
slot already holds max_pending_bytes, is refused at once with a status (LEX_ELIMIT or
LEX_ENOMEM) instead of being queued; it completes with no tokens.
Whenever a slot is free, every request that has arrived and fits joins one batch: the
payloads are gathered into the slot's pinned stage, copied to the device in one transfer,
scanned by one lex_run_batch, and the outputs copied back into pinned memory, all on the
slot's stream; an event marks completion.  Requests arriving meanwhile wait for the next
free slot, so batches on different slots overlap on the device.  A request's latency runs
from its arrival to the moment its result is in pinned host memory.
"""
from __future__ import annotations

import argparse
import gc
import json
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import abi
from .lexer import DOC_DTYPE, DOC_RESULT_DTYPE, Batch, Lexer


_SMALL = 8  # batches up to this many requests are gathered and split request by request


@dataclass
class Request:
    rid: int
    inst: int
    payload: np.ndarray          # uint8
    arrival: float               # seconds (scheduler clock)
    admitted: float = 0.0
    done: float = 0.0
    kinds: np.ndarray | None = None
    lens: np.ndarray | None = None
    ntokens: int = 0
    error_offset: int = 0
    status: int = 0


@dataclass
class _Slot:
    stream: object
    data: object
    kinds: object
    lens: object
    docs: object
    res: object
    total: object
    ws: object
    stage_in: object             # pinned uint8
    stage_docs: object           # pinned uint8 (DOC_DTYPE records)
    out_kinds: object            # pinned uint8
    out_lens: object             # pinned int32
    out_res: object              # pinned uint8 (DOC_RESULT_DTYPE records)
    out_total: object            # pinned int64[3]
    event: object = None
    batch: list = field(default_factory=list)


class Server:
    """K slots over one lex_batch; see the module notes."""

    def __init__(self, instances, budget_bytes: int = 16 << 30, slots: int = 4, max_docs: int = 8192,
                 lane_bytes: int = 1024, device: int = 0, slot_cap: int = 16 << 20,
                 max_pending_bytes: int | None = None):
        import torch

        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.batch = Batch(instances)
        self.opts = abi.RunOpts(lane_bytes=lane_bytes)
        self.max_docs = max_docs
        # a slot admits up to slot_bytes of input; its device memory (input and worst-case
        # output, document records and results, workspace) counts against the budget
        per_slot = budget_bytes // slots
        n = min(slot_cap, per_slot // 6) & ~15
        while n >= 4096 and self.slot_device_bytes(n) > per_slot:
            n = (n * 7 // 8) & ~15
        if n < 4096 or self.slot_device_bytes(n) > per_slot:
            raise ValueError("budget too small for the slots")
        self.slot_bytes = n
        self.reserved_bytes = slots * self.slot_device_bytes(n)
        self.budget_bytes = budget_bytes
        self.max_pending_bytes = max_pending_bytes if max_pending_bytes is not None else 8 * slots * n
        self.pending_bytes = 0
        self.refused: list[Request] = []
        self.max_busy = 0
        self.slots = []
        for _ in range(slots):
            ws_n = self.batch.workspace_size(max_docs, n, self.opts)
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(device=self.dev),
                data=torch.empty(n, dtype=torch.uint8, device=self.dev),
                kinds=torch.empty(n, dtype=torch.uint8, device=self.dev),
                lens=torch.empty(n, dtype=torch.int32, device=self.dev),
                docs=torch.empty(max_docs * 16, dtype=torch.uint8, device=self.dev),
                res=torch.empty(max_docs * 32, dtype=torch.uint8, device=self.dev),
                total=torch.zeros(3, dtype=torch.int64, device=self.dev),
                ws=torch.empty(ws_n, dtype=torch.uint8, device=self.dev),
                stage_in=torch.empty(n, dtype=torch.uint8, pin_memory=True),
                stage_docs=torch.empty(max_docs * 16, dtype=torch.uint8, pin_memory=True),
                out_kinds=torch.empty(n, dtype=torch.uint8, pin_memory=True),
                out_lens=torch.empty(n, dtype=torch.int32, pin_memory=True),
                out_res=torch.empty(max_docs * 32, dtype=torch.uint8, pin_memory=True),
                out_total=torch.zeros(3, dtype=torch.int64, pin_memory=True),
            ))
        self.pending: deque[Request] = deque()
        self.batch_sizes: list[int] = []

    def slot_device_bytes(self, n: int) -> int:
        """Device bytes of a slot of capacity n: input, kinds and lengths (6 n), document
        records and results (48 per document), and the batch workspace."""
        return 6 * n + 48 * self.max_docs + self.batch.workspace_size(self.max_docs, n, self.opts)

    # ------------------------------------------------------------- scheduling
    def admit(self, req: Request, now: float) -> bool:
        """Queues the request for the next free slot, or refuses it at once: LEX_ELIMIT when
        it is larger than a slot, LEX_ENOMEM when the queue already holds max_pending_bytes.
        A refused request completes (with its status, no tokens) at the next step."""
        req.admitted = now
        size = req.payload.size
        if size > self.slot_bytes or self.pending_bytes + size > self.max_pending_bytes:
            req.status = abi.LEX_ELIMIT if size > self.slot_bytes else abi.LEX_ENOMEM
            req.done = now
            req.kinds = np.zeros(0, np.uint8)
            req.lens = np.zeros(0, np.uint32)
            self.refused.append(req)
            return False
        self.pending.append(req)
        self.pending_bytes += size
        return True

    def busy(self) -> bool:
        return bool(self.pending) or bool(self.refused) or any(s.batch for s in self.slots)

    def _launch(self, slot: _Slot):
        torch = self.torch
        reqs, nbytes = [], 0
        while self.pending and len(reqs) < self.max_docs and nbytes + self.pending[0].payload.size <= self.slot_bytes:
            r = self.pending.popleft()
            reqs.append(r)
            nbytes += r.payload.size
        self.pending_bytes -= nbytes
        if not reqs:
            return
        docs = np.zeros(len(reqs), dtype=DOC_DTYPE)
        stage = slot.stage_in.numpy()
        if len(reqs) <= _SMALL:
            off = 0
            for i, r in enumerate(reqs):
                stage[off: off + r.payload.size] = r.payload
                docs[i] = (off, r.payload.size, r.inst, 0)
                off += r.payload.size
        else:  # the document table and the payload gather, one numpy call each
            sizes = np.fromiter((r.payload.size for r in reqs), dtype=np.uint64, count=len(reqs))
            docs["offset"][1:] = np.cumsum(sizes[:-1])
            docs["length"] = sizes
            docs["inst"] = np.fromiter((r.inst for r in reqs), dtype=np.uint32, count=len(reqs))
            off = int(sizes.sum())
            if off:
                np.concatenate([r.payload for r in reqs], out=stage[:off])
        slot.stage_docs.numpy()[: docs.nbytes] = docs.view(np.uint8)
        with torch.cuda.stream(slot.stream):
            slot.data[:off].copy_(slot.stage_in[:off], non_blocking=True)
            slot.docs[: docs.nbytes].copy_(slot.stage_docs[: docs.nbytes], non_blocking=True)
            self.batch.run_into(slot.data, off, slot.docs, len(reqs), slot.kinds, slot.lens, None, off, slot.res,
                                slot.total, slot.ws, self.opts, slot.stream)
            slot.out_kinds[:off].copy_(slot.kinds[:off], non_blocking=True)
            slot.out_lens[:off].copy_(slot.lens[:off], non_blocking=True)
            slot.out_res[: len(reqs) * 32].copy_(slot.res[: len(reqs) * 32], non_blocking=True)
            slot.out_total.copy_(slot.total, non_blocking=True)
            slot.event = torch.cuda.Event()
            slot.event.record(slot.stream)
        slot.batch = reqs
        self.batch_sizes.append(len(reqs))

    def _complete(self, slot: _Slot, now: float, done: list):
        res = slot.out_res.numpy()[: len(slot.batch) * 32].view(DOC_RESULT_DTYPE)
        kinds, lens = slot.out_kinds.numpy(), slot.out_lens.numpy()
        if len(slot.batch) <= _SMALL:
            for r, d in zip(slot.batch, res):
                a, b = int(d["tok_offset"]), int(d["tok_offset"] + d["ntokens"])
                r.kinds = kinds[a:b].copy()
                r.lens = lens[a:b].view(np.uint32).copy()
                r.ntokens, r.error_offset, r.status = int(d["ntokens"]), int(d["error_offset"]), int(d["status"])
                r.done = now
                done.append(r)
        else:
            # one copy of the batch's tokens out of the pinned buffers (the slot's next batch
            # reuses them); each request then holds views of it
            ntok = int(res["tok_offset"][-1] + res["ntokens"][-1])
            kinds = kinds[:ntok].copy()
            lens = lens[:ntok].view(np.uint32).copy()
            lo = res["tok_offset"].tolist()
            nt, eo, stt = res["ntokens"].tolist(), res["error_offset"].tolist(), res["status"].tolist()
            for i, r in enumerate(slot.batch):
                r.kinds = kinds[lo[i]: lo[i] + nt[i]]
                r.lens = lens[lo[i]: lo[i] + nt[i]]
                r.ntokens, r.error_offset, r.status = nt[i], eo[i], stt[i]
                r.done = now
                done.append(r)
        slot.batch = []
        slot.event = None

    def step(self, now_fn) -> list:
        """Completes finished slots and launches batches on free ones; returns the requests
        completed in this step."""
        done = self.refused
        self.refused = []
        for s in self.slots:
            if s.batch and s.event.query():
                self._complete(s, now_fn(), done)
        for s in self.slots:
            if not s.batch and self.pending:
                self._launch(s)
        self.max_busy = max(self.max_busy, sum(1 for s in self.slots if s.batch))
        return done


def make_pool(per_set: int, seed: int, median: int = 8192, sigma: float = 1.5, lo: int = 64, hi: int = 4 << 20):
    """Request payloads: per_set documents for each of C-like-L, C-like-D and JSON, log-normal
    sizes.  Returns a list of (instance, payload)."""
    import workloads

    sizes = workloads.lognormal_sizes(3 * per_set, median, sigma, lo, hi, workloads.substream(seed, 0))
    pool = []
    for i, n in enumerate(sizes):
        inst = i % 3
        n = int(n)
        if inst == 2:
            b = workloads.json(n, workloads.substream(seed, 100 + i))
        else:
            b = workloads.clike(n, workloads.substream(seed, 100 + i))
        pool.append((inst, np.array(b, copy=True)))
    return pool


def instances():
    from workloads import tokensets as T

    return [(Lexer.compile(T.as_tuples(T.CLIKE_L)), abi.LEX_MODE_EXACT),
            (Lexer.compile(T.as_tuples(T.CLIKE_D)), abi.LEX_MODE_DISCARD),
            (Lexer.compile(T.as_tuples(T.JSON)), abi.LEX_MODE_DISCARD)]


def open_loop(server: Server, pool, rate: float, seconds: float, seed: int, warmup: float = 0.0, keep=False):
    """Replays Poisson arrivals at `rate` per second for `seconds` against the wall clock
    (the first `warmup` seconds are not measured); returns metrics, and the completed
    requests when keep is set."""
    import workloads

    n = int(rate * seconds * 1.2) + 16
    gaps = workloads.exponential(n, rate, workloads.substream(seed, 1))
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < seconds]
    picks = (workloads.uniform(arrivals.size, workloads.substream(seed, 2)) * len(pool)).astype(np.int64)
    # the cyclic collector is paused while requests are timed: a full collection over the
    # completed requests would stall the scheduler for tens of milliseconds (reference
    # counting still frees everything this loop drops)
    gc_was = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        nxt, completed = 0, []
        while nxt < arrivals.size or server.busy():
            now = clock()
            while nxt < arrivals.size and arrivals[nxt] <= now:
                inst, payload = pool[picks[nxt]]
                server.admit(Request(nxt, inst, payload, float(arrivals[nxt])), now)
                nxt += 1
            completed += server.step(clock)
        wall = clock()
    finally:
        if gc_was:
            gc.enable()
    refused = [r for r in completed if r.arrival >= warmup and r.status in (abi.LEX_ELIMIT, abi.LEX_ENOMEM)]
    meas = [r for r in completed if r.arrival >= warmup and r.status not in (abi.LEX_ELIMIT, abi.LEX_ENOMEM)]
    lat = np.array([r.done - r.arrival for r in meas]) * 1e6
    wait = np.array([r.admitted - r.arrival for r in meas]) * 1e6
    nbytes = sum(r.payload.size for r in meas)
    span = max(1e-9, min(wall, seconds) - warmup)
    out = {
        "rate_per_s": rate, "seconds": seconds, "requests": len(meas),
        "p50_us": round(float(np.percentile(lat, 50)), 1) if lat.size else None,
        "p99_us": round(float(np.percentile(lat, 99)), 1) if lat.size else None,
        "admission_wait_p50_us": round(float(np.percentile(wait, 50)), 1) if wait.size else None,
        "completed_gbs": round(nbytes / span / 1e9, 4),
        "batches": len(server.batch_sizes),
        "batch_size_p50": float(np.percentile(server.batch_sizes, 50)) if server.batch_sizes else 0,
        "batch_size_max": int(max(server.batch_sizes)) if server.batch_sizes else 0,
        "errors": int(sum(r.status != 0 for r in meas)),
        "refused": len(refused),
        "max_slots_busy": server.max_busy,
        "slot_bytes": server.slot_bytes,
        "reserved_device_bytes": server.reserved_bytes,
    }
    server.batch_sizes.clear()
    return (out, completed) if keep else out


def main():
    ap = argparse.ArgumentParser(description="open-loop serving run (one JSON line per rate)")
    ap.add_argument("--rates", default="2000,10000,50000")
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--warmup", type=float, default=2.0)
    ap.add_argument("--pool", type=int, default=16384, help="documents per token set")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    pool = make_pool(args.pool, 7)
    server = Server(instances(), budget_bytes=int(args.budget_gib * (1 << 30)), slots=args.slots)
    for rate in (float(x) for x in args.rates.split(",")):
        print(json.dumps(open_loop(server, pool, rate, args.seconds, 6, args.warmup)), flush=True)


if __name__ == "__main__":
    main()
