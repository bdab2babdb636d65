"""GPU parity at the benchmark sizes, in the launch configuration bench.py times.

The 512 MiB C-like corpus (exact mode) and the 256 MiB JSON corpus (discard mode) are too
large for the oracle to lex whole in a test, so they are checked two ways:

* sampled stretches: at a certified byte c (LF), Theorem 1 (exact) and Theorem 3 (modulo
  I) make the input from c on lexable on its own, so the oracle lexes [c, c') for ~64 KiB
  stretches ending at a later LF, and the GPU's tokens starting inside the stretch must
  equal the oracle's, kind for kind and length for length;
* properties that hold at any size: in exact mode the lengths tile the input (their sum is
  the error offset), every length is positive and every kind in range; in discard mode the
  kept tokens are disjoint and in order.

The stray-byte variant of the C-like corpus overwrites one byte with 0x01 (the offset is
drawn from seed 3 and redrawn until the line holding it no longer lexes, the reading of
"injects" recorded in the design notes); its expected error offset is the oracle's, from
that line lexed alone (Corollary 1), and the output before the line must equal the clean
scan's.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu

N_CLIKE = 512 << 20
N_JSON = 256 << 20
STRETCH = 64 << 10
SAMPLES = 24


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def bench_opts():
    return P.RunOpts(chunk_bytes=64 << 10)  # as bench.py: 64 KiB chunks, lanes and path by default


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


def sampled_stretches(buf, starts, kinds, lens, oc, discard, seed):
    """Oracle on ~64 KiB stretches from random LFs against the GPU tokens starting there."""
    rng = np.random.default_rng(seed)
    n = buf.size
    for c in sorted(rng.integers(0, n - STRETCH, SAMPLES)):
        a = lf_after(buf, int(c))
        b = lf_after(buf, a + STRETCH)
        k, l, offs, con = oc.lex(bytes(buf[a:b]), discard=discard, offsets=True)
        assert con == b - a
        lo, hi = np.searchsorted(starts, a), np.searchsorted(starts, b)
        np.testing.assert_array_equal(kinds[lo:hi], k, err_msg=f"stretch [{a}, {b})")
        np.testing.assert_array_equal(lens[lo:hi], l, err_msg=f"stretch [{a}, {b})")
        np.testing.assert_array_equal(starts[lo:hi], offs.astype(np.int64) + a, err_msg=f"stretch [{a}, {b})")


@pytest.fixture(scope="module")
def clike_full():
    buf = workloads.clike(N_CLIKE, 2)
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
    buf, lx, oc, r, kinds, lens = clike_full
    assert r.status == 0 and r.error_offset == N_CLIKE
    assert r.nslices > 8000
    assert r.ntokens == kinds.size and lens.min() >= 1
    assert int(lens.sum(dtype=np.uint64)) == N_CLIKE  # exact mode: the tokens tile the input
    assert int(kinds.max()) < len(T.CLIKE_L)
    starts = np.zeros(lens.size, np.int64)
    np.cumsum(lens[:-1], out=starts[1:])
    sampled_stretches(buf, starts, kinds, lens, oc, False, seed=11)


def _stray(buf, oc, seed, want_error):
    """Overwrites buf (a copy) at draws from `seed` until the line holding the byte lexes
    (want_error False) or stops lexing (True); returns (buf, offset, line start, line end)."""
    for draw in range(200):
        x = workloads.stray_offset(buf.size, seed, draw)
        a = lf_before(buf, x)
        b = lf_after(buf, x + 1)  # an overwritten LF joins its line to the next
        line = bytearray(buf[a:b])
        line[x - a] = 1
        _, _, con = oc.lex(bytes(line))
        if (con < len(line)) == want_error:
            out = np.array(buf, copy=True)
            out[x] = 1
            return out, x, a, b, con
    raise AssertionError("no suitable draw")


@pytest.mark.parametrize("want_error", [True, False])
def test_clike_512mib_stray_byte(clike_full, want_error):
    buf, lx, oc, r, kinds, lens = clike_full
    bad, x, a, b, con = _stray(buf, oc, 3, want_error)
    print(f"[case] stray 0x01 at {x} (line [{a}, {b}), error={want_error})", flush=True)
    dev = torch.from_numpy(bad).cuda()
    rb = lx.run(dev, mode=P.LEX_MODE_EXACT, opts=bench_opts())
    del dev
    assert rb.status == 0
    gk = rb.kinds.cpu().numpy()
    gl = rb.lens.cpu().numpy().view(np.uint32)
    starts = np.zeros(lens.size, np.int64)
    np.cumsum(lens[:-1], out=starts[1:])
    before = int(np.searchsorted(starts, a))  # clean tokens before the line
    lk, ll, lcon = oc.lex(bytes(bad[a:b]))
    if want_error:
        # Corollary 1: everything before the line, then the line's tokens up to its halt
        assert rb.error_offset == a + lcon == a + con
        assert rb.ntokens == before + lk.size
    else:
        assert rb.error_offset == N_CLIKE and rb.ntokens == r.ntokens
    np.testing.assert_array_equal(gk[:before], kinds[:before])
    np.testing.assert_array_equal(gl[:before], lens[:before])
    np.testing.assert_array_equal(gk[before:before + lk.size], lk)
    np.testing.assert_array_equal(gl[before:before + lk.size], ll)


def test_json_256mib_discard():
    buf = workloads.json(N_JSON, 4)
    defs = T.as_tuples(T.JSON)
    lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
    dev = torch.from_numpy(buf).cuda()
    print(f"[case] JSON discard n={N_JSON} seed 4", flush=True)
    r = lx.run(dev, mode=P.LEX_MODE_DISCARD, offsets=True, opts=bench_opts())
    del dev
    assert r.status == 0 and r.error_offset == N_JSON
    assert r.nslices > 1000
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    starts = r.offsets.cpu().numpy()
    ws = [i for i, d in enumerate(T.JSON) if d.discard]
    assert not np.isin(kinds, ws).any() and lens.min() >= 1
    assert np.all(starts[1:] >= starts[:-1] + lens[:-1])  # kept tokens disjoint, in order
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
    starts = np.zeros(lens.size, np.int64)
    np.cumsum(lens[:-1], out=starts[1:])
    assert starts[-1] > (1 << 31)  # tokens past 2^31 bytes
    sampled_stretches(buf, starts, kinds, lens, oracle.OracleSet(defs), False, seed=12)


def test_batch_bench_workload_sampled():
    """The batched-documents workload at its benchmark size (50,000 documents, 2.53 GB, seed
    5: C-like-L exact, C-like-D discard, C-like-B discard, the last refused and hybrid
    planned), one lex_run_batch with default options (the batch's default lane for this
    size, 4 KiB).  Every document: token ranges are the exclusive prefix sum of the counts,
    nothing errs (the generator writes whole tokens), the totals agree.  Sampled documents,
    the largest of each instance among them, equal their oracle scan element by element."""
    insts = [(T.CLIKE_L, P.LEX_MODE_EXACT), (T.CLIKE_D, P.LEX_MODE_DISCARD), (T.CLIKE_B, P.LEX_MODE_DISCARD)]
    buf, offs, sizes, sets = workloads.docs(50000, 5)
    nd, n = sizes.size, buf.size
    batch = P.Batch([(P.Lexer.compile(T.as_tuples(d)), m) for d, m in insts])
    docs = np.zeros(nd, dtype=P.DOC_DTYPE)
    docs["offset"], docs["length"], docs["inst"] = offs, sizes, sets
    print(f"[case] batch bench workload: {nd} docs, {n} B, default opts", flush=True)
    r = batch.run(torch.from_numpy(buf).cuda(), docs, offsets=True)
    assert r.status == 0 and r.nerrors == 0
    res = r.docs
    assert (res["status"] == 0).all() and (res["error_offset"] == sizes).all()
    cnt = res["ntokens"].astype(np.uint64)
    want_off = np.zeros(nd, np.uint64)
    np.cumsum(cnt[:-1], out=want_off[1:])
    np.testing.assert_array_equal(res["tok_offset"], want_off)
    assert int(cnt.sum()) == r.ntokens and r.nslices > nd
    rng = np.random.default_rng(17)
    pick = set(rng.choice(nd, 300, replace=False).tolist())
    for k in range(len(insts)):
        of_k = np.flatnonzero(sets == k)
        pick.add(int(of_k[np.argmax(sizes[of_k])]))
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in insts]
    for i in sorted(pick):
        k, a, z = int(sets[i]), int(offs[i]), int(sizes[i])
        ok, ol, oo, con = orcs[k].lex(bytes(buf[a:a + z]), discard=bool(insts[k][1]), offsets=True)
        assert con == z, i
        t0, t1 = int(res["tok_offset"][i]), int(res["tok_offset"][i] + res["ntokens"][i])
        assert t1 - t0 == ok.size, i
        np.testing.assert_array_equal(r.kinds[t0:t1].cpu().numpy(), ok, err_msg=f"doc {i}")
        np.testing.assert_array_equal(r.lens[t0:t1].cpu().numpy().view(np.uint32), ol, err_msg=f"doc {i}")
        np.testing.assert_array_equal(r.offsets[t0:t1].cpu().numpy(), oo.astype(np.int64), err_msg=f"doc {i}")
