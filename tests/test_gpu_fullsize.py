"""GPU parity at the benchmark sizes, in the launch configuration bench.py times.

Every token of the benchmark configurations is compared with the oracle's, through the
digests ``tests/golden/stream_manifest.py`` wrote from the oracle alone (the serial
longest-match scan of Section 3, its own automata): the 512 MiB C-like corpus in exact
mode, both of its stray-byte variants (Corollary 1's truncation and error offset, or no
error when 0x01 lands where it is legal), the 256 MiB JSON corpus in modulo-I mode with
start offsets (Theorem 3), and all 50,000 documents of the batched workload.  The corpus
digest is checked first, so a drifted generator fails as such.  When a stream digest
differs, the test names the first block of 2^20 tokens (1,000 documents) whose digest
differs and re-lexes that region with the oracle from a certified LF (Theorem 1 and
Theorem 3 make the input from there lexable on its own), failing on the first token that
differs.

Properties that hold at any size are checked as well: in exact mode the lengths tile the
input, every length is positive and every kind in range; in discard mode the kept tokens
are disjoint and in order.  The 3 GiB case near the size limit has no manifest entry (the
oracle would take minutes); it keeps sampled stretches.
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

N_CLIKE = 512 << 20
N_JSON = 256 << 20
STRETCH = 64 << 10
SAMPLES = 24
MAN = SM.load()["cases"]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def bench_opts():
    return P.RunOpts(chunk_bytes=64 << 10)  # as bench.py: 64 KiB chunks, lanes and path by default


lf_after, lf_before = SM.lf_after, SM.lf_before


def compare_region(buf, starts, kinds, lens, oc, discard, a, b, what):
    """Oracle on [a, b) (a a certified LF boundary or 0) against the GPU tokens starting
    there, kind for kind, length for length and start for start."""
    k, l, offs, con = oc.lex(bytes(buf[a:b]), discard=discard, offsets=True)
    lo, hi = np.searchsorted(starts, a), np.searchsorted(starts, a + con)
    gk, gl, gs = kinds[lo:hi], lens[lo:hi], starts[lo:hi] - a
    m = min(gk.size, k.size)
    bad = np.flatnonzero((gk[:m] != k[:m]) | (gl[:m] != l[:m]) | (gs[:m] != offs[:m].astype(np.int64)))
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"{what}: first differing token {lo + i} at byte {a + int(offs[i])}: "
                             f"GPU (kind {gk[i]}, len {gl[i]}, start {a + gs[i]}) against oracle "
                             f"(kind {k[i]}, len {l[i]}, start {a + int(offs[i])})")
    assert gk.size == k.size, f"{what}: {gk.size} GPU tokens in [{a}, {a + con}), oracle {k.size}"


def sampled_stretches(buf, starts, kinds, lens, oc, discard, seed):
    """Oracle on ~64 KiB stretches from random LFs against the GPU tokens starting there."""
    rng = np.random.default_rng(seed)
    n = buf.size
    for c in sorted(rng.integers(0, n - STRETCH, SAMPLES)):
        a = lf_after(buf, int(c))
        b = lf_after(buf, a + STRETCH)
        compare_region(buf, starts, kinds, lens, oc, discard, a, b, f"stretch [{a}, {b})")


def starts_of(lens):
    s = np.zeros(lens.size, np.int64)
    if lens.size:
        np.cumsum(lens[:-1], out=s[1:])
    return s


def check_stream(want, buf, kinds, lens, starts, offsets, oc, discard, what):
    """The whole stream against the manifest's digests; on a difference, the first block
    whose digest differs is re-lexed by the oracle to name the first differing token."""
    got = SM.stream_digest(kinds, lens, offsets)
    same = got["kinds"] == want["kinds"] and got["lens"] == want["lens"]
    if offsets is not None:
        same = same and got["offsets"] == want["offsets"]
    if same and kinds.size == want["ntokens"]:
        return
    b = max(0, SM.first_bad_block(want["blocks"], got["blocks"]))
    t0 = min(b * SM.BLOCK_TOKENS, max(kinds.size - 1, 0))
    x0 = int(starts[t0]) if kinds.size else 0
    a = lf_before(buf, x0)
    end = int(starts[min(kinds.size - 1, t0 + SM.BLOCK_TOKENS)]) if kinds.size else buf.size
    compare_region(buf, starts, kinds, lens, oc, discard, a, lf_after(buf, max(end, x0 + 1)),
                   f"{what}, block {b}")
    raise AssertionError(f"{what}: digests differ from the oracle's (first differing block {b}, "
                         f"{kinds.size} tokens against {want['ntokens']}) but the block re-lexed equal")


@pytest.fixture(scope="module")
def clike_full():
    case = MAN["clike_512mib"]
    buf = SM.corpus(case)
    assert SM.sha(buf) == case["corpus_sha256"], "C-like corpus generator drifted"
    defs = T.as_tuples(T.CLIKE_L)
    lx = P.Lexer.compile(defs)
    dev = torch.from_numpy(buf).cuda()
    print(f"[case] C-like-L exact n={N_CLIKE} seed 2", flush=True)
    r = lx.run(dev, mode=P.LEX_MODE_EXACT, opts=bench_opts())
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    del dev
    return buf, lx, oracle.OracleSet(defs), r, kinds, lens


def test_clike_512mib_exact(clike_full):
    """Every token of the 512 MiB benchmark corpus equals the oracle's (whole-stream digests)."""
    buf, lx, oc, r, kinds, lens = clike_full
    want = MAN["clike_512mib"]
    assert r.status == 0 and r.error_offset == want["error_offset"] == N_CLIKE
    assert r.ntokens == want["ntokens"] == kinds.size
    assert r.nslices > 8000
    assert lens.min() >= 1 and int(lens.sum(dtype=np.uint64)) == N_CLIKE  # the tokens tile the input
    assert int(kinds.max()) < len(T.CLIKE_L)
    starts = starts_of(lens)
    check_stream(want, buf, kinds, lens, starts, None, oc, False, "C-like 512 MiB")
    sampled_stretches(buf, starts, kinds, lens, oc, False, seed=11)


@pytest.mark.parametrize("name", ["clike_512mib_stray_error", "clike_512mib_stray_ok"])
def test_clike_512mib_stray_byte(clike_full, name):
    """A stray 0x01 (the manifest's draw from seed 3): the whole output, token count and
    error offset equal the oracle's scan of the modified corpus (Corollary 1)."""
    buf, lx, oc, r, kinds, lens = clike_full
    want = MAN[name]
    x = want["stray_offset"]
    assert workloads.stray_offset(buf.size, want["stray_seed"], want["stray_draw"]) == x
    bad = np.array(buf, copy=True)
    bad[x] = 1
    assert SM.sha(bad) == want["stray_corpus_sha256"]
    print(f"[case] stray 0x01 at {x} ({name})", flush=True)
    dev = torch.from_numpy(bad).cuda()
    rb = lx.run(dev, mode=P.LEX_MODE_EXACT, opts=bench_opts())
    del dev
    assert rb.status == 0
    assert rb.error_offset == want["error_offset"] and rb.ntokens == want["ntokens"]
    if want["want_error"]:
        assert want["error_offset"] < N_CLIKE and want["error_offset"] <= x
    else:
        assert want["error_offset"] == N_CLIKE
    gk = rb.kinds.cpu().numpy()
    gl = rb.lens.cpu().numpy().view(np.uint32)
    assert int(gl.sum(dtype=np.uint64)) == rb.error_offset  # tokens tile [0, con)
    check_stream(want, bad, gk, gl, starts_of(gl), None, oc, False, name)


def test_json_256mib_discard():
    """Every kept token (kind, length, start offset) of the 256 MiB JSON corpus equals the
    oracle's modulo-I stream (Theorem 3)."""
    want = MAN["json_256mib"]
    buf = SM.corpus(want)
    assert SM.sha(buf) == want["corpus_sha256"], "JSON corpus generator drifted"
    defs = T.as_tuples(T.JSON)
    lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
    dev = torch.from_numpy(buf).cuda()
    print(f"[case] JSON discard n={N_JSON} seed 4", flush=True)
    r = lx.run(dev, mode=P.LEX_MODE_DISCARD, offsets=True, opts=bench_opts())
    del dev
    assert r.status == 0 and r.error_offset == want["error_offset"] == N_JSON
    assert r.ntokens == want["ntokens"]
    assert r.nslices > 1000
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    starts = r.offsets.cpu().numpy()
    ws = [i for i, d in enumerate(T.JSON) if d.discard]
    assert not np.isin(kinds, ws).any() and lens.min() >= 1
    assert np.all(starts[1:] >= starts[:-1] + lens[:-1])  # kept tokens disjoint, in order
    check_stream(want, buf, kinds, lens, starts, starts, oc, True, "JSON 256 MiB")
    sampled_stretches(buf, starts, kinds, lens, oc, True, seed=12)


def test_clike_3gib_exact():
    """Near the size limit: a 3 GiB (plus a ragged 77 bytes) C-like corpus, past 2^31 bytes,
    in the bench's launch configuration; the same tiling properties and sampled stretches."""
    n = (3 << 30) + 77
    buf = workloads.clike(n, 5)
    defs = T.as_tuples(T.CLIKE_L)
    lx = P.Lexer.compile(defs)
    dev = torch.from_numpy(buf).cuda()
    print(f"[case] C-like-L exact n={n} seed 5", flush=True)
    r = lx.run(dev, mode=P.LEX_MODE_EXACT, opts=bench_opts())
    del dev
    assert r.status == 0 and r.error_offset == n and r.nslices > 40000
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    del r
    torch.cuda.empty_cache()
    assert lens.min() >= 1 and int(lens.sum(dtype=np.uint64)) == n
    assert int(kinds.max()) < len(T.CLIKE_L)
    starts = starts_of(lens)
    assert starts[-1] > (1 << 31)  # tokens past 2^31 bytes
    sampled_stretches(buf, starts, kinds, lens, oracle.OracleSet(defs), False, seed=12)


def test_batch_bench_workload_whole():
    """The batched-documents workload at its benchmark size (50,000 documents, 2.53 GB, seed
    5: C-like-L exact, C-like-D discard, C-like-B discard, the last refused and hybrid
    planned), one lex_run_batch with default options (the batch's default lane for this
    size).  Every document's token count, error offset and tokens (kind, length, start
    offset relative to the document) equal the oracle's scan of that document alone, by the
    manifest's digests; token ranges are the exclusive prefix sum of the counts.  On a
    difference the first block of 1,000 documents whose digest differs is re-lexed by the
    oracle document by document."""
    want = MAN["docs_50k"]
    insts = [(T.NAMED[s], m) for s, m in zip(want["sets"], want["modes"])]
    buf, offs, sizes, sets = SM.corpus(want)
    assert SM.sha(buf) == want["corpus_sha256"], "batch corpus generator drifted"
    nd, n = sizes.size, buf.size
    batch = P.Batch([(P.Lexer.compile(T.as_tuples(d)), m) for d, m in insts])
    docs = np.zeros(nd, dtype=P.DOC_DTYPE)
    docs["offset"], docs["length"], docs["inst"] = offs, sizes, sets
    print(f"[case] batch bench workload: {nd} docs, {n} B, default opts", flush=True)
    r = batch.run(torch.from_numpy(buf).cuda(), docs, offsets=True)
    assert r.status == 0 and r.nerrors == want["incomplete_documents"]
    res = r.docs
    assert (res["status"] == 0).all()
    cnt = res["ntokens"].astype(np.uint64)
    want_off = np.zeros(nd, np.uint64)
    np.cumsum(cnt[:-1], out=want_off[1:])
    np.testing.assert_array_equal(res["tok_offset"], want_off)
    assert int(cnt.sum()) == r.ntokens == want["total_tokens"] and r.nslices > nd
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    starts = r.offsets.cpu().numpy()
    del r
    got = SM.docs_digest(cnt, res["error_offset"], kinds, lens, starts)
    if all(got[k] == want[k] for k in ("ntokens", "error_offsets", "kinds", "lens", "offsets")):
        return
    b = max(0, SM.first_bad_block(want["blocks"], got["blocks"]))
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in insts]
    for i in range(b * SM.DOC_BLOCK, min(nd, (b + 1) * SM.DOC_BLOCK)):
        k, a, z = int(sets[i]), int(offs[i]), int(sizes[i])
        ok, ol, oo, con = orcs[k].lex(bytes(buf[a:a + z]), discard=bool(insts[k][1]), offsets=True)
        t0, t1 = int(res["tok_offset"][i]), int(res["tok_offset"][i] + res["ntokens"][i])
        assert int(res["error_offset"][i]) == con, f"doc {i}: error offset"
        assert t1 - t0 == ok.size, f"doc {i}: {t1 - t0} tokens, oracle {ok.size}"
        np.testing.assert_array_equal(kinds[t0:t1], ok, err_msg=f"doc {i}")
        np.testing.assert_array_equal(lens[t0:t1], ol, err_msg=f"doc {i}")
        np.testing.assert_array_equal(starts[t0:t1], oo.astype(np.int64), err_msg=f"doc {i}")
    raise AssertionError(f"batch digests differ from the oracle's (first differing block {b}) "
                         f"but its documents re-lexed equal")
