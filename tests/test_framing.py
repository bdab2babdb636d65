"""Framing at the producer (Section 7.1): a reserved byte r is taken out of every token and
given a kind of its own.  CPU only: the oracle's framed set is pinned here to the paper's
claim about Table 2's block-comment row, to a brute-force sweep, to a framed tokenizer on
Python's ``re`` engine, and to the unframed scan; then the library's framed compile is held
to the oracle's certificates.
"""
import random

import numpy as np
import pytest

import oracle
import pyref
import workloads
from workloads import tokensets as T

RS = 0x1E


def _tuples(defs):
    return T.as_tuples(defs)


def test_block_comment_row_certifies_the_reserved_byte():
    """Table 2's block-comment row certifies nothing in either mode; framed by 0x1E it
    certifies that byte in both (Section 7.1), and every other byte stays refused."""
    defs = _tuples(T.TABLE2_ROW4_BCOMMENT)
    plain = oracle.OracleSet(defs).cert()
    assert plain["exact"] == frozenset() and plain["discard"] == frozenset()
    fr = oracle.OracleSet(defs, reserved=RS).cert()
    assert fr["exact"] == fr["discard"] == frozenset({RS})
    assert fr["exact_raw"] == fr["discard_raw"] == frozenset({RS})


def test_framed_c_like_b_certifies_the_reserved_byte():
    defs = _tuples(T.CLIKE_B)
    fr = oracle.OracleSet(defs, reserved=RS).cert()
    assert RS in fr["exact"] and RS in fr["discard"]


@pytest.mark.parametrize("defs,alpha", [
    (T.TABLE2_ROW4_BCOMMENT, b"/*a \n\x1e"),
    (T.CLIKE_B, b'/*"a\n\x1e'),
])
def test_framed_bruteforce_sweep(defs, alpha):
    """Every string over the alphabet up to length 6: splitting at every certified byte
    (0x1E included) reproduces the serial stream, and the lemma and theorem checks hold."""
    st = oracle.OracleSet(_tuples(defs), reserved=RS).bruteforce(alpha, 6)
    assert st["strings"] > 0 and st["mode_splits"] > 0
    for k, v in st.items():
        if k.endswith("_viol"):
            assert v == 0, (k, v)


@pytest.mark.parametrize("defs,alpha", [
    (T.CLIKE_B, b'a1 \n/*"\\\x1e'),
    (T.TABLE2_ROW4_BCOMMENT, b"a/* \n\x1e"),
    (T.JSON, b'"\\u0a1-.e \ntrue{}:,\x1e'),
])
def test_framed_oracle_vs_re(defs, alpha):
    """The oracle's framed lexer against the framed set written from its languages on
    Python's re engine (kind k keeps its words without r, kind len(defs) is r alone)."""
    tup = _tuples(defs)
    s = oracle.OracleSet(tup, reserved=RS)
    ref = pyref.compile_defs(tup)
    rng = random.Random(RS + len(tup))
    for _ in range(500):
        w = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 14)))
        k, l, con = s.lex(w)
        rt, rcon = pyref.lex_framed(ref, w, RS)
        assert con == rcon, w
        assert list(zip(k.tolist(), l.tolist())) == rt, w


def test_framed_equals_unframed_on_documents_without_r():
    """Without the reserved byte in the input the two sets scan alike (kind ids included:
    the reserved kind comes last)."""
    defs = _tuples(T.CLIKE_B)
    w = workloads.clike(1 << 16, 31, bcomment=True)
    assert not (w == RS).any()
    a = oracle.OracleSet(defs).lex(w)
    b = oracle.OracleSet(defs, reserved=RS).lex(w)
    assert a[2] == b[2] == w.size
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def _insert(w, at):
    out = bytearray()
    prev = 0
    for p in at:
        out += w[prev:p]
        out.append(RS)
        prev = p
    out += w[prev:]
    return bytes(out)


@pytest.mark.parametrize("defs", [T.CLIKE_B, T.CLIKE_L, T.JSON])
def test_producer_framing_reproduces_the_stream(defs):
    """A producer that writes r only at token boundaries of the unframed scan: the framed
    scan is the unframed stream with one r token at each inserted place, and the chunked
    scan cut at every r reproduces it."""
    tup = _tuples(defs)
    if defs is T.JSON:
        w = bytes(workloads.json(1 << 14, 5))
    else:
        w = bytes(workloads.clike(1 << 14, 5, bcomment=defs is T.CLIKE_B))
    plain = oracle.OracleSet(tup)
    k0, l0, o0, con0 = plain.lex(w, offsets=True)
    assert con0 == len(w)
    rng = random.Random(7)
    picks = sorted(rng.sample(range(o0.size), o0.size // 5))
    at = [int(o0[i]) for i in picks] + [len(w)]  # a separator at the very end too
    fw = _insert(w, at)
    fr = oracle.OracleSet(tup, reserved=RS)
    k1, l1, o1, con1 = fr.lex(fw, offsets=True)
    assert con1 == len(fw)
    rs_kind = len(tup)
    is_rs = k1 == rs_kind
    assert int(is_rs.sum()) == len(at) and (l1[is_rs] == 1).all()
    np.testing.assert_array_equal(k1[~is_rs], k0)
    np.testing.assert_array_equal(l1[~is_rs], l0)
    # the separators sit where the producer put them
    want = np.array(at, np.uint64) + np.arange(len(at), dtype=np.uint64)
    np.testing.assert_array_equal(o1[is_rs], want)
    cuts = [int(p) for p in np.flatnonzero(np.frombuffer(fw, np.uint8) == RS) if 0 < p < len(fw)]
    kc, lc, err = fr.lex_chunked(fw, cuts)
    assert err == len(fw)
    np.testing.assert_array_equal(kc, k1)
    np.testing.assert_array_equal(lc, l1)
    # modulo I with the separator declared discarded: the unframed image pi_I (Section 5)
    kd0, ld0, _ = plain.lex(w, discard=True)
    kd1, ld1, _ = oracle.OracleSet(tup, reserved=RS, reserved_discard=True).lex(fw, discard=True)
    np.testing.assert_array_equal(kd1, kd0)
    np.testing.assert_array_equal(ld1, ld0)
    kd2, _, _ = fr.lex(fw, discard=True)  # kept: one r token per separator
    assert int((kd2 == rs_kind).sum()) == len(at) and kd2.size == kd0.size + len(at)


def test_r_anywhere_still_splits_exactly():
    """Certification is static (Section 7.1): with r also inside comments and strings (a
    producer that failed to escape it) the chunked scan cut at every r still equals the
    serial scan of the framed set, malformed remainders included (Corollary 1)."""
    tup = _tuples(T.CLIKE_B)
    fr = oracle.OracleSet(tup, reserved=RS)
    rng = np.random.default_rng(11)
    for trial in range(6):
        w = workloads.clike(1 << 13, 40 + trial, bcomment=True).copy()
        pos = rng.choice(w.size, size=40, replace=False)
        w[pos] = RS
        k, l, con = fr.lex(w)
        cuts = [int(p) for p in np.flatnonzero(w == RS) if p > 0]
        kc, lc, err = fr.lex_chunked(w, cuts)
        assert err == con
        np.testing.assert_array_equal(kc, k)
        np.testing.assert_array_equal(lc, l)
        # no token but the reserved kind holds r
        offs = np.concatenate([[0], np.cumsum(l.astype(np.int64))[:-1]]) if l.size else np.zeros(0, np.int64)
        for kk, o, ln in zip(k, offs, l):
            if kk != len(tup):
                assert RS not in w[o:o + ln]


def test_generator_frames_at_token_boundaries():
    """workloads.clike(frame=k) opens records with r at token boundaries: deleting the
    separators gives a document whose unframed scan is the framed scan without them."""
    tup = _tuples(T.CLIKE_B)
    w = workloads.clike(1 << 15, 9, bcomment=True, frame=3)
    nrs = int((w == RS).sum())
    assert nrs > 50 and w[0] == RS
    k1, l1, con1 = oracle.OracleSet(tup, reserved=RS).lex(w)
    assert con1 == w.size
    is_rs = k1 == len(tup)
    assert int(is_rs.sum()) == nrs
    k0, l0, con0 = oracle.OracleSet(tup).lex(w[w != RS])
    assert con0 == w.size - nrs
    np.testing.assert_array_equal(k1[~is_rs], k0)
    np.testing.assert_array_equal(l1[~is_rs], l0)
