"""The library's packed tables, walked by a host model of the lane loop, against the oracle
(CPU only).  Catches table-packing mistakes before any GPU run: every token set, random
inputs (valid and corrupted), serial and split at certified bytes, both modes."""
import random

import numpy as np

import hostmodel
import oracle
import paper_2608_03473_amd as P
import workloads
from workloads import tokensets as T

from randsets import rand_set


def _check(defs, inputs, rng):
    lx = P.Lexer.compile(defs)
    oc = oracle.OracleSet(defs)
    for mode in (P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD):
        m = hostmodel.Model(lx, mode)
        cert = lx.cert(mode)
        for w in inputs:
            k, l, offs, con = oc.lex(w, discard=bool(mode), offsets=True)
            want = list(zip(k.tolist(), l.tolist(), offs.tolist()))
            got, err = m.scan(w, [])
            assert (got, err) == (want, con), (defs, w, mode)
            occ = [i for i in range(1, len(w)) if w[i] in cert]
            for cuts in (occ, sorted(rng.sample(occ, len(occ) // 2)) if occ else []):
                got, err = m.scan(w, cuts)
                assert (got, err) == (want, con), (defs, w, mode, cuts)


def test_random_sets_random_strings():
    rng = random.Random(1)
    for seed in range(150):
        defs = rand_set(seed, "abc")
        inputs = [bytes(rng.choice(b"abc") for _ in range(rng.randint(0, 12))) for _ in range(25)]
        _check(defs, inputs, rng)


def _corrupt(buf: bytes, rng, k=3):
    b = bytearray(buf)
    for _ in range(k):
        b[rng.randrange(len(b))] = rng.choice([0x01, ord("&"), ord('"'), ord("/"), ord("*"), ord(".")])
    return bytes(b)


def test_config_sets_on_corpora():
    rng = random.Random(2)
    cl = bytes(workloads.clike(3000, 11))
    clb = bytes(workloads.clike(3000, 12, bcomment=True))
    js = bytes(workloads.json(3000, 13))
    for defs, base in ((T.CLIKE_L, cl), (T.CLIKE_D, cl), (T.CLIKE_B, clb), (T.JSON, js)):
        inputs = [base[:600], base[600:1900]] + [_corrupt(base[:800], rng) for _ in range(6)]
        _check(T.as_tuples(defs), inputs, rng)


def test_nonmonotone_fallback_cases():
    """Longest match falls back to the last accepting position (JSON '1.', '1e+', '/' vs '/*')."""
    rng = random.Random(3)
    js = T.as_tuples(T.JSON)
    _check(js, [b"1.", b"1.5e", b"-1e+", b"1.x", b"[1.,2]", b"tru", b"\"a\\u12\"", b"1e5.", b"\n1.e\n"], rng)
    cb = T.as_tuples(T.CLIKE_B)
    _check(cb, [b"/*a", b"/* a\nb */", b"a/*b*/c", b"/**/", b"/*/", b"x /* y", b"//a\n/*"], rng)
    assert not P.Lexer.compile(js).info()["monotone"]


def test_windowed_emit_model():
    """The windowed emit's bookkeeping (window checkpoints, owner lookup, tiles, staged
    flush) restated on the host gives the oracle's tokens: monotone sets whose token ends are
    all counted, both planners' slice conventions, several lane lengths, buffer alignments
    and stage sizes (small stages force the direct path), and inputs with long tokens that
    leave lanes empty."""
    long_tok = b"x = 1;\n/* " + b"c" * 3000 + b" */\ny = 2;\n" + b"s = \"" + b"q" * 700 + b"\";\nz;\n"
    cases = [("clike_l", bytes(workloads.clike(20000, 3)), 0),
             ("clike_l", bytes(workloads.clike(3000, 4)) + long_tok + bytes(workloads.clike(3000, 5)), 0),
             ("log", bytes(workloads.loglines(12000, 37)), 0),
             ("clike_d", bytes(workloads.clike(9000, 6)), 0),
             ("clike_d", bytes(workloads.clike(9000, 6)), 1),
             ("clike_d", bytes(workloads.clike(3000, 4)) + long_tok.replace(b"/*", b"//") + bytes(workloads.clike(3000, 5)), 1)]
    for name, w, mode in cases:
        defs = T.as_tuples(T.NAMED[name])
        lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
        m = hostmodel.Model(lx, mode)
        k, l, offs, con = oc.lex(w, discard=bool(mode), offsets=True)
        want = (k.tolist(), l.tolist(), offs.tolist())
        cert = lx.cert(mode)
        for lane in (64, 256, 1024, 1 << 20):
            cuts = hostmodel.plan_cuts(w, cert, lane)
            plans = [(cuts[:-1], cuts[1:]), hostmodel.plan_fused(w, cert, lane)]
            for starts, ends in plans:
                for base in (0, 3, 63, 64, 100):
                    for stage in (1280, 150):
                        got = hostmodel.windowed(m, w, starts, ends, lane, base, 4, stage)
                        assert got == want, (name, lane, base, stage)
                        # without offsets: a discarding mode stages lengths
                        got = hostmodel.windowed(m, w, starts, ends, lane, base, 4, stage, offsets=False)
                        assert got == want[:2] + (None,), (name, mode, lane, base, stage)
        # a slice that halts: the windowed emit stands down
        bad = w[:3000] + b"\x01" + w[3000:]
        if oc.lex(bad, discard=bool(mode))[2] < len(bad):
            cuts = hostmodel.plan_cuts(bad, cert, 256)
            assert hostmodel.windowed(m, bad, cuts[:-1], cuts[1:], 256, 0) is None


def test_hybrid_plan_model():
    """The hybrid plan for refused token sets (speculative lanes with a common-token-start
    sync), restated on the host: whenever it cuts, every cut is a token start of the serial
    scan and the slices lexed from their cuts concatenate to the serial scan; it falls back
    (no cuts) on inputs whose serial scan halts and when a block comment longer than the
    sync window (2 KiB) spans a lane boundary."""
    defs = T.as_tuples(T.CLIKE_B)
    lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
    m = hostmodel.Model(lx, P.LEX_MODE_DISCARD)
    assert not lx.cert(P.LEX_MODE_DISCARD)  # refused: no useful certified byte
    split = 0
    for seed in range(10):
        w = bytes(workloads.clike([30000, 70000][seed % 2], 700 + seed, bcomment=True))
        if seed % 5 == 4:  # a stray byte; the draw may land where 0x01 is legal
            w = w[:len(w) // 3] + b"\x01" + w[len(w) // 3:]
        ke, le, oe, con = oc.lex(w, discard=False, offsets=True)
        cuts = hostmodel.spec_plan(m, w, 4096, 2048)
        if cuts is None:
            continue
        split += 1
        assert con == len(w), seed  # a plan that cuts never covers a halting scan
        assert set(cuts) <= set(oe.tolist()) | {0}, seed
        kd, ld, od, _ = oc.lex(w, discard=True, offsets=True)
        got = []
        for a, b in zip(cuts, cuts[1:] + [len(w)]):
            k, l, o, c = oc.lex(w[a:b], discard=True, offsets=True)
            assert c == b - a
            got += list(zip(k.tolist(), l.tolist(), (o + a).tolist()))
        assert got == list(zip(kd.tolist(), ld.tolist(), od.tolist())), seed
    assert split >= 8
    # the batch's parameters (S = X = 2 KiB) and its four-part walks of each slice: every part
    # start is a serial token start, and the parts lexed alone concatenate to the serial scan
    parted = 0
    for seed in range(6):
        w = bytes(workloads.clike([20000, 50000][seed % 2], 900 + seed, bcomment=True))
        cuts = hostmodel.spec_plan(m, w, 2048, 2048)
        if cuts is None:
            continue
        kd, ld, od, _ = oc.lex(w, discard=True, offsets=True)
        serial_starts = set(oc.lex(w, discard=False, offsets=True)[2].tolist())
        got = []
        for ps, (s0, e0) in zip(hostmodel.spec_parts(m, w, 2048, cuts), zip(cuts, cuts[1:] + [len(w)])):
            assert ps == sorted(ps) and all(s0 <= p <= e0 for p in ps)
            assert all(p in serial_starts or p == e0 for p in ps[1:]), seed
            parted += sum(1 for p in ps[1:] if s0 < p < e0)
            for a, b in zip(ps, ps[1:] + [e0]):
                k, l, o, c = oc.lex(w[a:b], discard=True, offsets=True)
                assert c == b - a
                got += list(zip(k.tolist(), l.tolist(), (o + a).tolist()))
        assert got == list(zip(kd.tolist(), ld.tolist(), od.tolist())), seed
    assert parted > 20
    # malformed: the serial scan halts, so the plan falls back
    w = bytearray(workloads.clike(30000, 9, bcomment=True))
    w[12000:12002] = b"@@"
    if oc.lex(bytes(w), discard=True)[2] < len(w):
        assert hostmodel.spec_plan(m, bytes(w), 4096, 2048) is None
    # the last token (a run of padding LFs, one whitespace token) spans the last lane's start:
    # the previous lane takes the rest and the plan still cuts
    w = bytes(workloads.clike(8100, 12, bcomment=True)) + b"\n" * 300
    cuts = hostmodel.spec_plan(m, w, 4096, 2048)
    assert cuts is not None and cuts[-1] == len(w)
    kd = oc.lex(w, discard=True, offsets=True)
    got = []
    for a, b in zip(cuts, cuts[1:] + [len(w)]):
        k, l, o, c = oc.lex(w[a:b], discard=True, offsets=True)
        got += list(zip(k.tolist(), l.tolist(), (o + a).tolist()))
    assert got == list(zip(kd[0].tolist(), kd[1].tolist(), kd[2].tolist()))
    # a block comment of 5000 bytes across the boundary at 4096: no common start in 2048 bytes
    w = bytes(workloads.clike(3000, 10)) + b"\n/* " + b"x" * 5000 + b" */\n" + bytes(workloads.clike(6000, 11))
    assert oc.lex(w, discard=True)[2] == len(w)
    assert hostmodel.spec_plan(m, w, 4096, 2048) is None


def test_failed_lookahead_memo():
    """Bounded failed lookahead (the Θ(N²) pathology of naive longest match, removed by
    remembering failed (state, position) pairs as Reps does): the fallback keeps up to four
    failed traces as cursors and stops a re-scan that meets one.  Same tokens as the oracle
    with any number of cursors; linear work on the paper's a^N example over {a, a+b, ;} and
    on unterminated block comments, where plain re-scans are quadratic."""
    rng = random.Random(4)
    for seed in range(120):
        defs = rand_set(seed, "abc")
        lx = P.Lexer.compile(defs)
        if lx.info()["monotone"]:
            continue
        oc = oracle.OracleSet(defs)
        m = hostmodel.Model(lx, P.LEX_MODE_EXACT)
        for _ in range(12):
            w = bytes(rng.choice(b"abc") for _ in range(rng.randint(0, 40)))
            k, l, offs, con = oc.lex(w, offsets=True)
            want = (list(zip(k.tolist(), l.tolist(), offs.tolist())), None if con == len(w) else con)
            for memo in (0, 1, 2, 4):
                assert m.walk(w, 0, len(w), memo=memo) == want, (defs, w, memo)

    ex = [("a", 0, False), ("a+b", 0, False), (";", 0, False)]
    m = hostmodel.Model(P.Lexer.compile(ex), P.LEX_MODE_EXACT)
    for n in (400, 1600):
        w = b"a" * n
        plain, memo = [0], [0]
        got0, _ = m.walk(w, 0, n, memo=0, work=plain)
        got4, _ = m.walk(w, 0, n, memo=4, work=memo)
        assert got0 == got4 == [(0, 1, i) for i in range(n)]
        assert plain[0] > n * n // 4 and memo[0] < 6 * n, (n, plain[0], memo[0])

    cb = T.as_tuples(T.CLIKE_B)
    oc = oracle.OracleSet(cb)
    m = hostmodel.Model(P.Lexer.compile(cb), P.LEX_MODE_EXACT)
    for unit in (b"/*a", b"/*a\n", b'/* "x', b"/**a"):
        w = unit * 300
        k, l, offs, con = oc.lex(w, offsets=True)
        plain, memo = [0], [0]
        got0 = m.walk(w, 0, len(w), memo=0, work=plain)
        got4 = m.walk(w, 0, len(w), memo=4, work=memo)
        want = (list(zip(k.tolist(), l.tolist(), offs.tolist())), None if con == len(w) else con)
        assert got0 == got4 == want, unit
        assert memo[0] < 8 * len(w), (unit, plain[0], memo[0])


def test_windowed_emit_model_nonmonotone():
    """The windowed emit on non-monotone automata (framed C-like-B, JSON, exact mode): a scan
    in which no slice falls back walks the serial trace in every window, so the windowed
    emit's tokens are the oracle's; a scan with a fallback stands it down (the model returns
    None, the library runs the lane emit)."""
    fr = T.as_tuples(T.CLIKE_B)
    cases = [(P.Lexer.compile_framed(fr), oracle.OracleSet(fr, reserved=0x1E),
              bytes(workloads.clike(30000, 7, bcomment=True, frame=3))),
             (P.Lexer.compile(T.as_tuples(T.JSON)), oracle.OracleSet(T.as_tuples(T.JSON)),
              bytes(workloads.json(30000, 8)))]
    for lx, oc, w in cases:
        assert not lx.info()["monotone"]
        for mode in (P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD):
            m = hostmodel.Model(lx, mode)
            k, l, offs, con = oc.lex(w, discard=bool(mode), offsets=True)
            want = (k.tolist(), l.tolist(), offs.tolist())
            cert = lx.cert(mode)
            if not cert:
                continue
            for lane in (64, 1024):
                cuts = hostmodel.plan_cuts(w, cert, lane)
                for starts, ends in [(cuts[:-1], cuts[1:]), hostmodel.plan_fused(w, cert, lane)]:
                    for base in (0, 5, 70):
                        assert hostmodel.windowed(m, w, starts, ends, lane, base, 4, 1280) == want, lane
                        got = hostmodel.windowed(m, w, starts, ends, lane, base, 4, 1280, offsets=False)
                        assert got == want[:2] + (None,), (mode, lane)
    # a fallback inside a slice (an unterminated comment cut by a separator): stood down
    lx, oc, w = cases[0]
    bad = w[:5000] + b"/* x" + bytes([0x1E]) + w[5000:]
    cert = lx.cert(P.LEX_MODE_EXACT)
    cuts = hostmodel.plan_cuts(bad, cert, 256)
    assert hostmodel.windowed(hostmodel.Model(lx, P.LEX_MODE_EXACT), bad, cuts[:-1], cuts[1:], 256, 0) is None


def _token_string(oc, rng, pieces=120):
    """Words the oracle lexes as one token each, joined by ';' (certified, a kind of its
    own): a scan of it never falls back, since each word's longest match is the word."""
    words = []
    for _ in range(400):
        w = bytes(rng.choice(b"abc") for _ in range(rng.randint(1, 7)))
        k, l, con = oc.lex(w)
        if con == len(w) and len(k) == 1:
            words.append(w)
    if not words:
        return None
    return b";".join(rng.choice(words) for _ in range(pieces))


def test_windowed_emit_model_random_sets():
    """Random token sets (monotone or not) with a certified ';', exact mode, on strings long
    enough for many lanes: whenever no slice falls back, the windowed emit's tokens are the
    oracle's, else it stands down.  Strings of whole tokens give non-monotone sets scans
    without fallbacks; random strings give both outcomes."""
    rng = random.Random(6)
    ran = nonmono = disc = 0
    for seed in range(200):
        defs = rand_set(seed, "abc") + [(";", 0, False)]
        lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
        for mode in (P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD):
            cert = lx.cert(mode)
            if not cert:
                continue
            m = hostmodel.Model(lx, mode)
            for w in (_token_string(oc, rng), bytes(rng.choice(b"abc;") for _ in range(600))):
                if w is None:
                    continue
                k, l, offs, con = oc.lex(w, discard=bool(mode), offsets=True)
                if con < len(w):
                    continue
                want = (k.tolist(), l.tolist(), offs.tolist())
                for lane in (16, 64):
                    cuts = hostmodel.plan_cuts(w, cert, lane)
                    got = hostmodel.windowed(m, w, cuts[:-1], cuts[1:], lane, 7, offsets=False)
                    if got is not None:
                        ran += 1
                        nonmono += not lx.info()["monotone"]
                        disc += m.disc
                        assert got == want[:2] + (None,), (defs, mode, lane)
                        assert hostmodel.windowed(m, w, cuts[:-1], cuts[1:], lane, 7) == want, (defs, mode, lane)
    assert ran > 100 and nonmono > 20 and disc > 20, (ran, nonmono, disc)
