"""Whole-stream expected values for the benchmark workloads, written by the oracle.

``python tests/golden/stream_manifest.py [case ...]`` regenerates ``stream_manifest.json``
(every case, or only the named ones).  It calls
only ``oracle/`` (the serial longest-match scan of Section 3, per-kind NFAs) and
``workloads/`` (the seeded corpus generators), never the HIP library.  For every case it
records:

* the SHA-256 of the generated corpus, so a drifted generator is caught before any
  comparison (the CPU tests re-check these digests);
* the oracle's token count and error offset con(w) (Section 3; Corollary 1 on malformed
  input);
* SHA-256 digests of its whole output: kinds as u8, lengths as little-endian u32 and,
  where the scan reports them, start offsets as little-endian u64;
* short digests of consecutive blocks of tokens (documents, for the batch), so a
  comparison that fails can name the first block that differs.

The cases are the benchmark configurations: the 1 MiB and 512 MiB C-like corpora in exact
mode (seeds 1 and 2), both stray-byte variants of the 512 MiB corpus (seed 3: a draw whose
line stops lexing, and one where 0x01 lands inside a string or comment and is legal), the
256 MiB JSON corpus in modulo-I mode with offsets (seed 4), every document of the
50,000-document batch (seed 5), and the 512 MiB C-like corpus with block comments (seed 2)
in exact mode under the C-like-B set: framed (records of 8 lines opened by 0x1E, the set
framed by that byte, Section 7.1) and unframed (no certified byte: the hybrid plan).  The helpers below are shared with the GPU tests, which
digest the device's output the same way.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PATH = os.path.join(HERE, "stream_manifest.json")
BLOCK_TOKENS = 1 << 20  # tokens per block digest of a single stream
DOC_BLOCK = 1000        # documents per block digest of the batch

EXACT, DISCARD = 0, 1

# The benchmark workloads: generator, size and seed, token set and mode.
CASES = {
    "clike_1mib": dict(gen="clike", n=1 << 20, seed=1, set="clike_l", mode=EXACT),
    "clike_512mib": dict(gen="clike", n=512 << 20, seed=2, set="clike_l", mode=EXACT),
    "clike_512mib_stray_error": dict(gen="clike", n=512 << 20, seed=2, set="clike_l", mode=EXACT,
                                     stray_seed=3, want_error=True),
    "clike_512mib_stray_ok": dict(gen="clike", n=512 << 20, seed=2, set="clike_l", mode=EXACT,
                                  stray_seed=3, want_error=False),
    "json_256mib": dict(gen="json", n=256 << 20, seed=4, set="json", mode=DISCARD, with_offsets=True),
    "clikeb_512mib_framed": dict(gen="clike", n=512 << 20, seed=2, bcomment=True, frame=8, set="clike_b",
                                 reserved=0x1E, mode=EXACT),
    "clikeb_512mib": dict(gen="clike", n=512 << 20, seed=2, bcomment=True, frame=0, set="clike_b", mode=EXACT),
    "docs_50k": dict(gen="docs", count=50000, seed=5, sets=["clike_l", "clike_d", "clike_b"],
                     modes=[EXACT, DISCARD, DISCARD]),
}


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(memoryview(np.ascontiguousarray(a)).cast("B"))
    return h.hexdigest()


def _le(a, dt):
    return np.ascontiguousarray(a).astype(dt, copy=False)


def stream_digest(kinds, lens, offsets=None) -> dict:
    """Digests of one token stream: whole arrays, then blocks of BLOCK_TOKENS tokens."""
    k = _le(kinds, np.uint8)
    l = _le(lens, "<u4")
    d = {"kinds": sha(k), "lens": sha(l)}
    if offsets is not None:
        d["offsets"] = sha(_le(offsets, "<u8"))
    d["blocks"] = [sha(k[i:i + BLOCK_TOKENS], l[i:i + BLOCK_TOKENS])[:16]
                   for i in range(0, k.size, BLOCK_TOKENS)]
    return d


def docs_digest(ntok, err, kinds, lens, offsets) -> dict:
    """Digests of a batch: per-document counts and error offsets, the concatenated streams
    (documents in order), and blocks of DOC_BLOCK documents (their counts and tokens)."""
    nt = _le(ntok, "<u8")
    k, l, o = _le(kinds, np.uint8), _le(lens, "<u4"), _le(offsets, "<u8")
    ends = np.cumsum(nt.astype(np.uint64))
    blocks = []
    for i in range(0, nt.size, DOC_BLOCK):
        t0 = int(ends[i - 1]) if i else 0
        t1 = int(ends[min(nt.size, i + DOC_BLOCK) - 1])
        blocks.append(sha(nt[i:i + DOC_BLOCK], k[t0:t1], l[t0:t1], o[t0:t1])[:16])
    return {"ntokens": sha(nt), "error_offsets": sha(_le(err, "<u8")), "kinds": sha(k), "lens": sha(l),
            "offsets": sha(o), "total_tokens": int(ends[-1]) if nt.size else 0, "blocks": blocks}


def first_bad_block(want: list, got: list) -> int:
    for i, (a, b) in enumerate(zip(want, got)):
        if a != b:
            return i
    return min(len(want), len(got)) if len(want) != len(got) else -1


def lf_after(buf, x):
    """First LF at or after x (or len(buf))."""
    n = buf.size
    while x < n:
        hit = np.flatnonzero(buf[x:min(n, x + (1 << 20))] == 10)
        if hit.size:
            return x + int(hit[0])
        x += 1 << 20
    return n


def lf_before(buf, x):
    """Start of the line holding x: one past the last LF before x (or 0)."""
    while x > 0:
        lo = max(0, x - 4096)
        hit = np.flatnonzero(buf[lo:x] == 10)
        if hit.size:
            return lo + int(hit[-1]) + 1
        x = lo
    return 0


def corpus(case: dict, stray_offset: int | None = None):
    """The case's input bytes (for "docs": (bytes, offsets, sizes, set ids))."""
    import workloads
    if case["gen"] == "clike":
        buf = workloads.clike(case["n"], case["seed"], bcomment=case.get("bcomment", False),
                              frame=case.get("frame", 0))
        if stray_offset is not None:
            buf[stray_offset] = 1
        return buf
    if case["gen"] == "json":
        return workloads.json(case["n"], case["seed"])
    if case["gen"] == "docs":
        return workloads.docs(case["count"], case["seed"])
    raise ValueError(case["gen"])


def load() -> dict:
    with open(PATH) as f:
        return json.load(f)


# ---------------------------------------------------------------------------- writer
def _oracle_set(name, reserved=None):
    """The oracle's compilation of a named set; reserved: framed by that byte (Section 7.1)."""
    import oracle
    from workloads import tokensets as T
    return oracle.OracleSet(T.as_tuples(T.NAMED[name]), reserved=reserved)


def pick_stray(buf, oc, seed, want_error):
    """The first draw from `seed` whose overwritten line stops lexing (want_error) or still
    lexes (not want_error), judged by the oracle on that line alone: the line starts at a
    certified LF boundary, so by Theorem 1 its scan is the serial scan's there."""
    import workloads
    for draw in range(200):
        x = workloads.stray_offset(buf.size, seed, draw)
        a = lf_before(buf, x)
        b = lf_after(buf, x + 1)  # an overwritten LF joins its line to the next
        line = bytearray(buf[a:b])
        line[x - a] = 1
        _, _, con = oc.lex(bytes(line))
        if (con < len(line)) == want_error:
            return draw, x
    raise AssertionError("no suitable draw")


def _single(name):
    case = CASES[name]
    t0 = time.time()
    oc = _oracle_set(case["set"], case.get("reserved"))
    buf = corpus(case)
    out = {"corpus_sha256": sha(buf)}
    if "stray_seed" in case:
        draw, x = pick_stray(buf, oc, case["stray_seed"], case["want_error"])
        buf[x] = 1
        out.update(stray_draw=draw, stray_offset=x, stray_corpus_sha256=sha(buf))
    disc = case["mode"] == DISCARD
    if case.get("with_offsets"):
        k, l, o, con = oc.lex(buf, discard=disc, offsets=True)
    else:
        (k, l, con), o = oc.lex(buf, discard=disc), None
    out.update(ntokens=int(k.size), error_offset=int(con))
    out.update(stream_digest(k, l, o))
    out["oracle_seconds"] = round(time.time() - t0, 1)
    return name, out


def _doc_shard(args):
    lo, hi = args
    import workloads
    case = CASES["docs_50k"]
    sizes, sets = workloads.doc_plan(case["count"], case["seed"])
    ocs = [_oracle_set(s) for s in case["sets"]]
    ks, ls, os_, nt, er = [], [], [], [], []
    for i in range(lo, hi):
        s = int(sets[i])
        d = workloads.doc(case["seed"], i, int(sizes[i]), s)
        k, l, o, con = ocs[s].lex(d, discard=case["modes"][s] == DISCARD, offsets=True)
        ks.append(k), ls.append(l), os_.append(o), nt.append(k.size), er.append(con)
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return (lo, np.array(nt, np.uint64), np.array(er, np.uint64), cat(ks, np.uint8), cat(ls, np.uint32),
            cat(os_, np.uint64))


def _docs(pool, workers):
    case = CASES["docs_50k"]
    t0 = time.time()
    buf, offs, sizes, sets = corpus(case)
    head = {"corpus_sha256": sha(buf), "sizes_sha256": sha(_le(sizes, "<u8")), "sets_sha256": sha(sets),
            "nbytes": int(buf.size)}
    del buf
    n = case["count"]
    step = (n + workers * 4 - 1) // (workers * 4)
    parts = sorted(pool.map(_doc_shard, [(i, min(n, i + step)) for i in range(0, n, step)]), key=lambda p: p[0])
    nt = np.concatenate([p[1] for p in parts])
    er = np.concatenate([p[2] for p in parts])
    k = np.concatenate([p[3] for p in parts])
    l = np.concatenate([p[4] for p in parts])
    o = np.concatenate([p[5] for p in parts])
    head.update(docs_digest(nt, er, k, l, o))
    head["incomplete_documents"] = int((er != sizes).sum())
    head["oracle_seconds"] = round(time.time() - t0, 1)
    return "docs_50k", head


def main(names=None):
    """Write every case, or only `names`, keeping the other cases' recorded values."""
    from concurrent.futures import ProcessPoolExecutor
    sys.path.insert(0, ROOT)
    workers = min(8, os.cpu_count() or 1)
    names = list(CASES) if not names else names
    assert all(n in CASES for n in names), names
    keep = load()["cases"] if os.path.exists(PATH) and len(names) < len(CASES) else {}
    out = {"about": ("Written by tests/golden/stream_manifest.py from the oracle (serial longest-match "
                     "scan, Section 3; Corollary 1 on malformed input) over the seeded corpora of "
                     "workloads/; never from the HIP library."),
           "block_tokens": BLOCK_TOKENS, "doc_block": DOC_BLOCK, "cases": {}}
    out["cases"].update({k: v for k, v in keep.items() if k in CASES and k not in names})
    with ProcessPoolExecutor(workers) as pool:
        singles = [pool.submit(_single, name) for name in names if name != "docs_50k"]
        if "docs_50k" in names:
            name, d = _docs(pool, workers)
            out["cases"][name] = dict(CASES[name], **d)
        for f in singles:
            name, d = f.result()
            out["cases"][name] = dict(CASES[name], **d)
            print(f"{name}: {d['ntokens']} tokens, error offset {d['error_offset']}, "
                  f"{d['oracle_seconds']} s", flush=True)
    out["cases"] = {k: out["cases"][k] for k in CASES}
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {PATH}")


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main(sys.argv[1:])
