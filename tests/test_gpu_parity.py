"""GPU parity: the HIP path through the C ABI against the oracle, element by element.

Sizes the oracle finishes in seconds that still span many lanes, several 4 KiB bitmap
tiles and ragged tails; both planner paths; several lane lengths; both modes; malformed
inputs (Corollary 1's truncation and error offset); edge cases.  The bar is bit-exact
kinds, lengths, offsets, token count and error offset.
"""
import random

import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2608_03473_amd")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


_LEX, _ORC = {}, {}


def lexers(name):
    if name not in _LEX:
        defs = T.as_tuples(T.NAMED[name])
        _LEX[name] = P.Lexer.compile(defs)
        _ORC[name] = oracle.OracleSet(defs)
    return _LEX[name], _ORC[name]


def to_dev(buf, pad_front=0):
    a = np.asarray(buf, dtype=np.uint8)
    if not pad_front:
        return torch.from_numpy(a.copy()).cuda()
    big = torch.zeros(a.size + pad_front, dtype=torch.uint8, device="cuda")
    big[pad_front:] = torch.from_numpy(a.copy()).cuda()
    return big[pad_front:]


def check(name, buf, mode, opts=None, pad_front=0, offsets=True, label=""):
    lx, oc = lexers(name)
    print(f"[case] {name} mode={mode} n={len(buf)} opts={opts and (opts.lane_bytes, opts.path)} "
          f"pad={pad_front} {label}", flush=True)
    k, l, o, con = oc.lex(bytes(buf), discard=bool(mode & 1), offsets=True)
    r = lx.run(to_dev(buf, pad_front), mode=mode, offsets=offsets, opts=opts)
    assert r.status == 0
    assert r.error_offset == con, (r.error_offset, con)
    assert r.ntokens == len(k), (r.ntokens, len(k))
    np.testing.assert_array_equal(r.kinds.cpu().numpy(), k)
    np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l)
    if offsets:
        np.testing.assert_array_equal(r.offsets.cpu().numpy().astype(np.uint64), o)
    return r


def opts(lane, path, emit=0):
    return P.RunOpts(lane_bytes=lane, path=path, emit=emit)


CL = workloads.clike(1 << 20, 1)  # the 1 MiB config, seed 1


@pytest.mark.parametrize("emit", [P.LEX_EMIT_DEFAULT, P.LEX_EMIT_LANE])
@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("lane", [16, 48, 64, 256, 1024, 4096, 0])
def test_clike_1mib_exact(path, lane, emit):
    r = check("clike_l", CL, P.LEX_MODE_EXACT, opts(lane, path, emit))
    assert r.nslices > 1


@pytest.mark.parametrize("path", [1, 2, 3])
def test_windowed_dense_tokens_direct(path):
    """One-byte tokens: every wave's output range outgrows its LDS stage, so the windowed
    emit writes token by token."""
    dense = np.frombuffer(b"a;b;" * 50000 + b"\n" + b"x=1;" * 30000, np.uint8)
    for lane in (64, 1024):
        check("clike_l", dense, P.LEX_MODE_EXACT, opts(lane, path))


@pytest.mark.parametrize("pad", [0, 1, 63])
def test_windowed_lane_starts_on_tile_boundaries(pad):
    """A certified byte (LF) at every multiple of 4096 bytes: lanes start exactly where a
    64-window tile of the windowed emit begins, so the token ending there is closed by the
    previous tile's last window; with the buffer offset the boundaries shift."""
    b = np.array(CL[: 1 << 19], copy=True)
    b[4096::4096] = ord("\n")
    b[4096 * 3 - 1] = ord("\n")  # and one just before a boundary
    for lane in (64, 1024, 4096):
        for path in (1, 2, 3):
            check("clike_l", b, P.LEX_MODE_EXACT, opts(lane, path), pad_front=pad)


@pytest.mark.parametrize("tiles", [1, 2, 15, 16, 17, 255, 257, 1025])
def test_windowed_tile_counts(tiles):
    """Tile counts around the windowed emit's split: workgroups take equal ranges of 64-window
    tiles and their waves draw tiles one at a time from a counter in LDS, reading the first
    window of the adjacent tile for each.  Counts below, at and above a workgroup's waves and
    the number of workgroups, ragged (the last tile partial), at two buffer offsets."""
    n = tiles * 4096 - 100
    buf = workloads.clike(n, 700 + tiles)
    for pad in (0, 37):
        for path in (1, 2):
            check("clike_l", buf, P.LEX_MODE_EXACT, opts(0, path), pad_front=pad, offsets=pad == 0)
    check("clike_d", buf, P.LEX_MODE_DISCARD, opts(0, 2))


def test_windowed_long_slice_falls_back():
    """A slice of 2^24 bytes or more (one 17 MiB comment): its checkpoints cannot hold its
    counts, so the lane emit takes the scan (after the one-pass kernel, its fallback)."""
    big = np.concatenate([CL[:5000], np.frombuffer(b"// ", np.uint8),
                          np.full(17 << 20, ord("c"), np.uint8), np.frombuffer(b"\n", np.uint8), CL[:7000]])
    for path in (2, 3):
        check("clike_l", big, P.LEX_MODE_EXACT, opts(1024, path), offsets=False)


def sparse_lf(buf, keep_every, seed):
    """buf with most LFs (the only certified byte of C-like-L) turned into spaces: one in
    keep_every stays, so lanes often hold none and slices run across many lanes."""
    b = np.array(buf, copy=True)
    lf = np.flatnonzero(b == 10)
    rng = np.random.default_rng(seed)
    b[lf[rng.random(lf.size) >= 1.0 / keep_every]] = 32
    return b


def no_comments(buf):
    """buf with every line comment blanked to spaces (so that removing LFs later does not
    turn the following lines into comment text)."""
    _, oc = lexers("clike_l")
    kinds, lens, offs, _ = oc.lex(bytes(buf), offsets=True)
    lc = [i for i, d in enumerate(T.CLIKE_L) if d.name == "LCOMMENT"]
    b = np.array(buf, copy=True)
    sel = np.isin(kinds, lc)
    for o, n in zip(offs[sel], lens[sel]):
        b[o:o + n] = 32
    return b


def lf_at(buf, positions):
    """buf with an LF at each given position that lies inside an IDENT, INT or SPACE token
    of the oracle's scan (there an LF only splits the token and the input stays lexable; in
    a string, a comment or a two-byte operator it would not); returns the buffer and how
    many were placed."""
    _, oc = lexers("clike_l")
    kinds, lens, offs, _ = oc.lex(bytes(buf), offsets=True)
    safe = [i for i, d in enumerate(T.CLIKE_L) if d.name in ("IDENT", "INT", "SPACE")]
    ok = np.zeros(len(buf), bool)
    sel = np.isin(kinds, safe)
    for o, n in zip(offs[sel], lens[sel]):
        ok[o:o + n] = True
    b = np.array(buf, copy=True)
    placed = 0
    for x in positions:
        if 0 < x < b.size and ok[x]:
            b[x] = 10
            placed += 1
    return b, placed


@pytest.mark.parametrize("path", [1, 2, 3])
@pytest.mark.parametrize("lane", [128, 256, 1024])
def test_planner_edges(path, lane):
    """The fused planner's cases: lanes without a certified byte (empty slices), slices
    across many lanes, certified bytes exactly at lane targets and at 128-byte line
    boundaries, a slice ending at a lane target; aligned and unaligned buffers."""
    base = CL[:300000]
    for label, buf in [("sparse 1/60", sparse_lf(base, 60, 1)), ("sparse 1/400", sparse_lf(base, 400, 2)),
                       ("no LF", sparse_lf(base[:20000], 10 ** 9, 3))]:
        for pad in (0, 5, 77):
            check("clike_l", buf, P.LEX_MODE_EXACT, opts(lane, path), pad_front=pad, label=label)
    sp = sparse_lf(no_comments(base), 200, 4)
    at = [j * lane + d for j in range(1, sp.size // lane) for d in (-1, 0, 1, 127, 128)]
    at_buf, placed = lf_at(sp, at)
    assert placed > sp.size // lane
    for pad in (0, 64, 3):
        check("clike_l", at_buf, P.LEX_MODE_EXACT, opts(lane, path), pad_front=pad, label="LF at targets")


@pytest.mark.parametrize("path", [1, 2, 3])
def test_clike_ragged_and_unaligned(path):
    for n in (1, 15, 16, 17, 63, 64, 65, 4095, 4097, 70001):
        for pad in (0, 3):
            check("clike_l", CL[:n], P.LEX_MODE_EXACT, opts(16, path), pad_front=pad)


def test_serial_mode_and_empty():
    check("clike_l", CL[:200000], P.LEX_MODE_SERIAL)
    r = check("clike_l", CL[:0], P.LEX_MODE_EXACT)
    assert r.ntokens == 0 and r.error_offset == 0


def _stray(buf, k, seed):
    b = np.array(buf, copy=True)
    rng = random.Random(seed)
    for _ in range(k):
        b[rng.randrange(b.size)] = 0x01
    return b


@pytest.mark.parametrize("path", [1, 2, 3])
def test_malformed_error_offset(path):
    """Corollary 1: output truncated at the first halting slice, error offset = con(w)."""
    base = CL[:300000]
    for seed in range(8):
        for lane in (16, 256):
            check("clike_l", _stray(base, 1 + seed % 3, seed), P.LEX_MODE_EXACT, opts(lane, path), label=f"seed{seed}")
    # an unterminated string and a lone '&'
    for bad in (b'x = "abc\ny', b"a && b & c\n", b"\x01", b"ok\n\x01"):
        buf = np.frombuffer(bytes(CL[:5000]) + bad + bytes(CL[5000:9000]), np.uint8)
        check("clike_l", buf, P.LEX_MODE_EXACT, opts(64, path))


@pytest.mark.parametrize("path", [1, 2, 3])
def test_discard_clike_d(path):
    check("clike_d", CL, P.LEX_MODE_DISCARD, opts(256, path))
    check("clike_d", CL, P.LEX_MODE_EXACT, opts(256, path))  # empty exact map: one slice


@pytest.mark.parametrize("path", [1, 2, 3])
def test_json_discard(path):
    js = workloads.json(2 << 20, 4)
    r = check("json", js, P.LEX_MODE_DISCARD, opts(128, path))
    assert r.nslices > 100
    check("json", js[:300000], P.LEX_MODE_EXACT, opts(128, path))  # refused: one lane
    # non-monotone fallbacks inside many lanes
    bad = np.frombuffer(b"\n".join([b"1.", b"[1.5e]", b"-", b"1e+", b"tru", b"{\"a\": 1.}"] * 50), np.uint8)
    check("json", bad, P.LEX_MODE_DISCARD, opts(16, path))
    # kinds and lengths only (the lane emit's packed walk), fallbacks included
    check("json", js, P.LEX_MODE_DISCARD, opts(256, path), offsets=False)
    check("json", bad, P.LEX_MODE_DISCARD, opts(16, path), offsets=False)


def test_clike_b_refused():
    """C-like-B has no useful certified byte.  Buffers longer than one speculative lane are
    split by the hybrid plan (and must still equal the serial scan); it falls back to one
    slice when the serial scan halts or a block comment longer than the sync window spans a
    lane boundary; serial mode and short buffers are one slice."""
    cb = workloads.clike(400000, 9, bcomment=True)
    r = check("clike_b", cb, P.LEX_MODE_DISCARD)
    assert r.nslices > 50
    r = check("clike_b", cb, P.LEX_MODE_DISCARD | P.LEX_MODE_SERIAL)
    assert r.nslices == 1
    check("clike_b", np.frombuffer(b"/* a\nb */ x /* y", np.uint8), P.LEX_MODE_DISCARD)
    bad = np.array(cb[:100000], copy=True)
    bad[70000:70002] = ord("@")
    check("clike_b", bad, P.LEX_MODE_DISCARD, label="halting")
    long_comment = np.concatenate([workloads.clike(3000, 11), np.frombuffer(b"\n/* " + b"x" * 5000 + b" */\n", np.uint8),
                                   workloads.clike(60000, 12)])
    r = check("clike_b", long_comment, P.LEX_MODE_DISCARD, label="long comment across a lane boundary")
    assert r.nslices == 1
    for n in (4097, 4096 + 600, 9000):
        check("clike_b", cb[:n], P.LEX_MODE_DISCARD, pad_front=3, label="just over one lane")
    tail = np.concatenate([workloads.clike(8100, 13, bcomment=True), np.full(300, 10, np.uint8)])
    r = check("clike_b", tail, P.LEX_MODE_DISCARD, label="last token across the last lane's start")
    assert r.nslices == 2


def test_clike_b_refused_exact_windowed():
    """The same hybrid-plan cases in exact mode, where every token end is counted: the
    windowed emit runs over the hybrid cuts (a non-monotone automaton: it stands down for a
    scan in which a slice fell back, and the lane emit writes the tokens)."""
    lx, _ = lexers("clike_b")
    cb = workloads.clike(400000, 9, bcomment=True)
    plan = lx.plan(cb.size, P.LEX_MODE_EXACT)
    assert plan["hybrid"] == 1 and plan["windowed"] == 1
    r = check("clike_b", cb, P.LEX_MODE_EXACT, label="hybrid, windowed")
    assert r.nslices > 50
    check("clike_b", cb, P.LEX_MODE_EXACT, offsets=False, label="hybrid, windowed, no offsets")
    bad = np.array(cb[:100000], copy=True)
    bad[70000:70002] = ord("@")
    check("clike_b", bad, P.LEX_MODE_EXACT, label="halting")
    long_comment = np.concatenate([workloads.clike(3000, 11), np.frombuffer(b"\n/* " + b"x" * 5000 + b" */\n", np.uint8),
                                   workloads.clike(60000, 12)])
    r = check("clike_b", long_comment, P.LEX_MODE_EXACT, label="long comment across a lane boundary")
    assert r.nslices == 1
    for n in (4097, 4096 + 600, 9000):
        check("clike_b", cb[:n], P.LEX_MODE_EXACT, pad_front=3, label="just over one lane")
    tail = np.concatenate([workloads.clike(8100, 13, bcomment=True), np.full(300, 10, np.uint8)])
    r = check("clike_b", tail, P.LEX_MODE_EXACT, label="last token across the last lane's start")
    assert r.nslices == 2
    # unterminated comments cut by lane boundaries: fallbacks inside slices
    w = np.frombuffer(b"/*a" * 3000, np.uint8)  # the oracle re-scans naively: kept short
    check("clike_b", w, P.LEX_MODE_EXACT, label="fallbacks in every slice")


def test_log_planning_workload():
    w = workloads.loglines(1 << 20, 40)
    r = check("log", w, P.LEX_MODE_EXACT, opts(1024, 1))
    assert r.ntokens == 2 * ((1 << 20) // 40) + 1


def test_overflow_status():
    lx, oc = lexers("clike_l")
    k, l, con = oc.lex(bytes(CL[:10000]))
    r = lx.run(to_dev(CL[:10000]), cap=len(k) - 1)
    assert r.status == P.LEX_EOVERFLOW and r.ntokens == len(k)
    r = lx.run(to_dev(CL[:10000]), cap=len(k))
    assert r.status == 0 and r.ntokens == len(k)


def test_cert_bitmap_kernel():
    lx, _ = lexers("json")
    js = workloads.json(100003, 3)
    bits = lx.cert_bitmap(to_dev(js), P.LEX_MODE_DISCARD).cpu().numpy().view(np.uint64)
    want = np.isin(js, [9, 10, 13])
    got = np.unpackbits(bits.view(np.uint8), bitorder="little")[: js.size].astype(bool)
    np.testing.assert_array_equal(got, want)


def test_random_sets_short_strings():
    """Random token sets (the brute-force family) on short strings, one scan per string."""
    from randsets import rand_set
    rng = random.Random(4)
    for seed in range(30):
        defs = rand_set(seed, "abc")
        lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
        for _ in range(12):
            w = bytes(rng.choice(b"abc") for _ in range(rng.randint(1, 40)))
            for mode in (0, 1):
                k, l, con = oc.lex(w, discard=bool(mode))
                r = lx.run(to_dev(np.frombuffer(w, np.uint8)), mode=mode, opts=opts(16, 1 + (seed & 1)))
                assert r.error_offset == con and r.ntokens == len(k), (defs, w, mode)
                np.testing.assert_array_equal(r.kinds.cpu().numpy(), k)
                np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l)


def test_random_sets_many_lanes():
    """Random token sets (monotone or not) with a certified ';' on strings of whole tokens
    (no fallback: the windowed emit also serves non-monotone sets there) and on random
    strings (fallbacks and halts: the lane emit), split into many lanes on every path."""
    from randsets import rand_set
    rng = random.Random(9)
    for seed in range(60):
        defs = rand_set(seed, "abc") + [(";", 0, False)]
        lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
        words = []
        for _ in range(300):
            w = bytes(rng.choice(b"abc") for _ in range(rng.randint(1, 7)))
            k, _, con = oc.lex(w)
            if con == len(w) and len(k) == 1:
                words.append(w)
        inputs = [bytes(rng.choice(b"abc;") for _ in range(3000))]
        if words:
            inputs.append(b";".join(rng.choice(words) for _ in range(700)))
        for w in inputs:
            for mode in (0, 1):
                k, l, o, con = oc.lex(w, discard=bool(mode), offsets=True)
                for path in (1, 2, 3):
                    print(f"[case] random set {seed} n={len(w)} mode={mode} path={path}", flush=True)
                    r = lx.run(to_dev(np.frombuffer(w, np.uint8)), mode=mode, offsets=True, opts=opts(16, path))
                    assert r.status == 0 and r.error_offset == con and r.ntokens == len(k), (defs, mode, path)
                    np.testing.assert_array_equal(r.kinds.cpu().numpy(), k)
                    np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l)
                    np.testing.assert_array_equal(r.offsets.cpu().numpy().astype(np.uint64), o)


@pytest.mark.parametrize("path", [0, 1, 2])
def test_graph_replays_single_buffer(path):
    """One lex_run captured in a hipGraph (its launches use no memset and allocate nothing)
    and replayed several times, with other eager scans and synchronisations in between:
    every replay equals the eager scan."""
    lx, _ = lexers("clike_l")
    buf = workloads.clike((4 << 20) + 77, 31)
    n = buf.size
    o = opts(0, path)
    data = to_dev(buf)
    kinds = torch.empty(n, dtype=torch.uint8, device="cuda")
    lens = torch.empty(n, dtype=torch.int32, device="cuda")
    res = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(lx.workspace_size(n, 0, o), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    lx.run_into(data, n, 0, kinds, lens, None, n, res, ws, o, stream)
    torch.cuda.synchronize()
    want_res = res.cpu().clone()
    nt = int(want_res[0])
    want_k, want_l = kinds[:nt].cpu().clone(), lens[:nt].cpu().clone()
    print(f"[case] graph replays, path {path}, {nt} tokens", flush=True)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.graph(graph, stream=side):
        lx.run_into(data, n, 0, kinds, lens, None, n, res, ws, o, torch.cuda.current_stream())
    other = to_dev(workloads.clike(1 << 20, 32))
    for rep in range(3):
        kinds.zero_()
        lens.zero_()
        res.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(res.cpu(), want_res), rep
        assert torch.equal(kinds[:nt].cpu(), want_k) and torch.equal(lens[:nt].cpu(), want_l), rep
        # eager work between replays, on other buffers
        r = lx.run(other, mode=0)
        assert r.status == 0
        torch.cuda.synchronize()
