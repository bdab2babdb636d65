"""GPU parity of framed scans (Section 7.1): a C-like-B set framed by the reserved byte 0x1E,
compiled by lex_compile_framed, scanned through the C ABI single-buffer and batched, against
the oracle's framed set, element by element; at the benchmark's 512 MiB size, framed and
unframed, every token against the whole-stream digests the oracle wrote.  The framed set
certifies 0x1E, so a framed document takes the certified planner (several slices, no hybrid
plan), where the unframed set is refused.  The bar is bit-exact kinds, lengths, offsets,
token count and error offset.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import stream_manifest as SM  # noqa: E402

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu

RS = 0x1E
DEFS = T.as_tuples(T.CLIKE_B)


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def sets():
    return {
        "lx": P.Lexer.compile_framed(DEFS),
        "lx_disc": P.Lexer.compile_framed(DEFS, reserved_discard=True),
        "oc": oracle.OracleSet(DEFS, reserved=RS),
        "oc_disc": oracle.OracleSet(DEFS, reserved=RS, reserved_discard=True),
    }


def check(lx, oc, buf, mode, opts=None, label="", offsets=True):
    print(f"[case] framed C-like-B mode={mode} n={len(buf)} "
          f"opts={opts and (opts.lane_bytes, opts.path)} offsets={offsets} {label}", flush=True)
    k, l, o, con = oc.lex(bytes(buf), discard=bool(mode & 1), offsets=True)
    r = lx.run(torch.from_numpy(np.array(buf, np.uint8, copy=True)).cuda(), mode=mode, offsets=offsets, opts=opts)
    assert r.status == 0
    assert r.error_offset == con, (r.error_offset, con)
    assert r.ntokens == len(k), (r.ntokens, len(k))
    np.testing.assert_array_equal(r.kinds.cpu().numpy(), k)
    np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l)
    if offsets:
        np.testing.assert_array_equal(r.offsets.cpu().numpy().astype(np.uint64), o)
    return r


DOC = workloads.clike((1 << 20) + 333, 21, bcomment=True, frame=4)  # ragged tail


@pytest.mark.parametrize("mode", [P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD])
@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("lane", [64, 1024, 0])
def test_framed_document_splits_at_the_separator(sets, mode, path, lane):
    lx, oc = sets["lx"], sets["oc"]
    plan = lx.plan(DOC.size, mode, P.RunOpts(lane_bytes=lane, path=path))
    assert plan["hybrid"] == 0
    # the windowed emit in both modes, on this non-monotone automaton (no slice of this
    # document falls back; modulo I its staged words carry lengths)
    assert plan["windowed"] == 1 and plan["path"] in (1, 2)
    r = check(lx, oc, DOC, mode, P.RunOpts(lane_bytes=lane, path=path))
    assert r.nslices > 1
    assert int((r.kinds.cpu().numpy() == len(DEFS)).sum()) == int((DOC == RS).sum())


@pytest.mark.parametrize("mode", [P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD])
@pytest.mark.parametrize("path", [1, 2])
def test_framed_without_offsets(sets, mode, path):
    """Kinds and lengths only: the lane emit's packed walk (no branch per byte), which
    non-monotone automata take with the last accepting step tracked and the fallback after
    each block; separators anywhere, so comments and strings are cut and fall back."""
    lx, oc = sets["lx"], sets["oc"]
    r = check(lx, oc, DOC, mode, P.RunOpts(lane_bytes=256, path=path), offsets=False)
    assert r.nslices > 1
    rng = np.random.default_rng(8)
    w = workloads.clike(400000, 14, bcomment=True).copy()
    w[rng.choice(w.size, 900, replace=False)] = RS
    check(lx, oc, w, mode, P.RunOpts(lane_bytes=64, path=path), "separator anywhere", offsets=False)


def test_separator_discarded(sets):
    """The separator declared discarded: the modulo-I stream has no separator tokens."""
    r = check(sets["lx_disc"], sets["oc_disc"], DOC, P.LEX_MODE_DISCARD, P.RunOpts(lane_bytes=256))
    assert r.nslices > 1 and not (r.kinds.cpu().numpy() == len(DEFS)).any()


def test_framed_edges(sets):
    """Separators at both ends and in runs, the separator alone, empty and tiny inputs, a
    separator inside comments and strings (a producer that failed to escape it), a stray
    byte (truncation at the right offset), and one long block comment between two
    separators (a slice far longer than a lane)."""
    lx, oc = sets["lx"], sets["oc"]
    mode = P.LEX_MODE_EXACT
    o = P.RunOpts(lane_bytes=64)
    check(lx, oc, np.zeros(0, np.uint8), mode, o, "empty")
    check(lx, oc, np.array([RS], np.uint8), mode, o, "separator alone")
    check(lx, oc, np.full(5000, RS, np.uint8), mode, o, "only separators")
    w = workloads.clike(20000, 3, bcomment=True, frame=1).copy()
    w[0] = w[-1] = RS
    w[100:110] = RS
    check(lx, oc, w, mode, o, "runs and ends")
    rng = np.random.default_rng(5)
    w = workloads.clike(300000, 4, bcomment=True).copy()
    w[rng.choice(w.size, 700, replace=False)] = RS
    check(lx, oc, w, mode, o, "separator anywhere")
    check(lx, oc, w, P.LEX_MODE_DISCARD, o, "separator anywhere, modulo I")
    w0 = workloads.clike(200000, 6, bcomment=True, frame=2)
    for p in range(150000, 151000):  # a stray byte outside comments and strings
        w = w0.copy()
        w[p] = 1
        if oc.lex(w)[2] < w.size:
            break
    r = check(lx, oc, w, mode, o, "stray byte")
    assert r.error_offset < w.size
    body = b"/*" + b"x\n" * 40000 + b"*/"
    w = np.frombuffer(bytes([RS]) + b"a b " + bytes([RS]) + body + bytes([RS]) + b" c\n" * 100, np.uint8)
    r = check(lx, oc, w, mode, o, "long comment between separators")
    # a cut is the first certified byte at or after a lane's target: the separator at 5
    # precedes the first target, so the one interior cut is the one after the comment
    assert r.nslices == 2


def test_framed_documents_batched(sets):
    """Framed and unframed documents in one batch, with the framed set and the unframed
    (refused, hybrid-planned) set as two instances: each document equals its oracle scan."""
    lx = sets["lx"]
    plain = P.Lexer.compile(DEFS)
    batch = P.Batch([(lx, P.LEX_MODE_EXACT), (plain, P.LEX_MODE_DISCARD)])
    orcs = [sets["oc"], oracle.OracleSet(DEFS)]
    rng = np.random.default_rng(12)
    parts, recs, off = [], [], 0
    for i in range(80):
        n = int(np.clip(np.exp(np.log(8192) + 1.5 * rng.standard_normal()), 0, 1 << 20))
        inst = i % 2
        b = workloads.clike(n, 500 + i, bcomment=True, frame=3 if inst == 0 else 0) if n else np.zeros(0, np.uint8)
        parts.append(np.array(b, copy=True))
        recs.append((off, n, inst, 0))
        off += n
    data = np.concatenate(parts)
    docs = np.array(recs, dtype=P.DOC_DTYPE)
    print(f"[case] framed batch of {docs.size} docs, {data.size} B", flush=True)
    r = batch.run(torch.from_numpy(data).cuda(), docs, offsets=True, opts=P.RunOpts(lane_bytes=1024))
    assert r.status == 0
    kinds, lens = r.kinds.cpu().numpy(), r.lens.cpu().numpy().view(np.uint32)
    offs = r.offsets.cpu().numpy()
    for i, (doc, res) in enumerate(zip(docs, r.docs)):
        inst = int(doc["inst"])
        w = bytes(data[doc["offset"]: doc["offset"] + doc["length"]])
        k, l, o, con = orcs[inst].lex(w, discard=inst == 1, offsets=True)
        assert res["status"] == 0 and res["error_offset"] == con, i
        a, b = int(res["tok_offset"]), int(res["tok_offset"] + res["ntokens"])
        assert b - a == len(k), i
        np.testing.assert_array_equal(kinds[a:b], k, err_msg=f"doc {i}")
        np.testing.assert_array_equal(lens[a:b], l, err_msg=f"doc {i}")
        np.testing.assert_array_equal(offs[a:b], o.astype(np.int64), err_msg=f"doc {i}")
        if inst == 0 and doc["length"] > 16384:
            assert res["nslices"] > 1, i


def test_framed_full_size_sampled(sets):
    """A 512 MiB framed C-like-B document, exact mode, as the benchmark's framed leg runs
    it: the separator count, the token count and sampled windows against the oracle."""
    n = 512 << 20
    lx, oc = sets["lx"], sets["oc"]
    host = workloads.clike(n, 2, bcomment=True, frame=8)
    print(f"[case] framed C-like-B full size n={n}", flush=True)
    r = lx.run(torch.from_numpy(host).cuda(), mode=P.LEX_MODE_EXACT, offsets=True)
    assert r.status == 0 and r.error_offset == n and r.nslices > 1000
    kinds = r.kinds.cpu().numpy()
    offs = r.offsets.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    is_rs = kinds == len(DEFS)
    seps = np.flatnonzero(host == RS)
    assert int(is_rs.sum()) == seps.size
    np.testing.assert_array_equal(offs[is_rs], seps.astype(np.int64))
    # sampled windows: from one separator to a later one, the oracle's scan of that window
    # is the device's tokens over it (0x1E is certified: a scan may start there)
    rng = np.random.default_rng(3)
    for j in rng.choice(seps.size - 40, 12, replace=False):
        a, b = int(seps[j]), int(seps[j + 40])
        k, l, con = oc.lex(bytes(host[a:b]))
        assert con == b - a
        i0, i1 = np.searchsorted(offs, [a, b])
        np.testing.assert_array_equal(kinds[i0:i1], k)
        np.testing.assert_array_equal(lens[i0:i1], l)


@pytest.mark.parametrize("name", ["clikeb_512mib_framed", "clikeb_512mib"])
def test_clikeb_512mib_whole(sets, name):
    """Every token of the benchmark's 512 MiB C-like-B scans, framed (the certified planner)
    and unframed (no certified byte: the hybrid plan), in the launch configuration the
    benchmark times (default plan, no offsets), against the oracle's whole-stream digests.
    On a difference the first block of 2^20 tokens that differs is named and, framed,
    re-lexed by the oracle from the separator before it to the one after it (0x1E is
    certified under the framed set, so a scan may start there, Theorem 1)."""
    want = SM.load()["cases"][name]
    framed = "reserved" in want
    n, mode = want["n"], P.LEX_MODE_EXACT
    host = SM.corpus(want)
    assert SM.sha(host) == want["corpus_sha256"], "C-like-B corpus generator drifted"
    lx = sets["lx"] if framed else P.Lexer.compile(DEFS)
    plan = lx.plan(n, mode)
    assert bool(plan["hybrid"]) != framed
    print(f"[case] {name} n={n} path={plan['path']} lane={plan['lane_bytes']} hybrid={plan['hybrid']}",
          flush=True)
    r = lx.run(torch.from_numpy(host).cuda(), mode=mode)
    assert r.status == 0 and r.error_offset == want["error_offset"] == n
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    got = SM.stream_digest(kinds, lens)
    if r.ntokens == want["ntokens"] and (got["kinds"], got["lens"]) == (want["kinds"], want["lens"]):
        return
    b = max(0, SM.first_bad_block(want["blocks"], got["blocks"]))
    msg = (f"{name}: digests differ from the oracle's (first differing block {b}, "
           f"{r.ntokens} tokens against {want['ntokens']})")
    if framed and kinds.size:
        starts = np.zeros(lens.size, np.int64)
        np.cumsum(lens[:-1], out=starts[1:])
        t0 = min(b * SM.BLOCK_TOKENS, kinds.size - 1)
        t1 = min(kinds.size - 1, t0 + SM.BLOCK_TOKENS)
        seps = np.flatnonzero(host == RS)
        i = np.searchsorted(seps, starts[t0], side="right")
        a = int(seps[i - 1]) if i else 0
        j = np.searchsorted(seps, starts[t1], side="right")
        e = int(seps[j]) if j < seps.size else n
        k, l, o, con = sets["oc"].lex(bytes(host[a:e]), offsets=True)
        lo, hi = np.searchsorted(starts, [a, a + con])
        gk, gl, gs = kinds[lo:hi], lens[lo:hi], starts[lo:hi] - a
        m = min(gk.size, k.size)
        bad = np.flatnonzero((gk[:m] != k[:m]) | (gl[:m] != l[:m]) | (gs[:m] != o[:m].astype(np.int64)))
        if bad.size:
            x = int(bad[0])
            msg += (f"; first differing token {lo + x} at byte {a + int(o[x])}: GPU (kind {gk[x]}, "
                    f"len {gl[x]}) against oracle (kind {k[x]}, len {l[x]})")
    raise AssertionError(msg)
