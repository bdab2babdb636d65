"""The library's token-set compiler (Glushkov + Hopcroft, its own certificate code) against
the oracle (Thompson + Moore, its own checker).  CPU only: lex_compile does not need a GPU.

Both trim to the live subautomaton and minimise, so the automata are isomorphic: state
counts, re-entrancy and all four maps (exact/modulo-I, raw/useful) must agree.
"""
import random

import numpy as np
import pytest

import oracle
import paper_2608_03473_amd as P
from workloads import tokensets as T

from randsets import rand_set

SETS = dict(T.NAMED)
SETS.update({k: getattr(T, k) for k in ("TABLE2_ROW1", "TABLE2_ROW2_STR", "TABLE2_ROW3_LCOMMENT",
                                        "TABLE2_ROW4_BCOMMENT", "TABLE2_BARRED", "TABLE2_LINE_BLOCK",
                                        "CLIKE_L_I", "CLIKE_L_BLOCK_I", "UTF8")})


def _agree(lx: P.Lexer, oc: dict, what):
    info = lx.info()
    assert info["q0_live"] == oc["q0_live_state"], what
    if oc["q0_live_state"]:
        assert info["nstates"] == oc["nstates"], what
        assert bool(info["reentrant"]) == oc["reentrant"], what
    assert lx.cert(P.LEX_MODE_EXACT) == oc["exact"], what
    assert lx.cert(P.LEX_MODE_DISCARD) == oc["discard"], what
    assert lx.cert(P.LEX_MODE_EXACT, raw=True) == oc["exact_raw"], what
    assert lx.cert(P.LEX_MODE_DISCARD, raw=True) == oc["discard_raw"], what


@pytest.mark.parametrize("name", sorted(SETS))
def test_named_sets(name):
    defs = T.as_tuples(SETS[name])
    _agree(P.Lexer.compile(defs), oracle.OracleSet(defs).cert(), name)


@pytest.mark.parametrize("reserved", [0x1E, 0x0A, 0x00, 0x2F, 0xFF])
@pytest.mark.parametrize("name", ["clike_b", "clike_l", "json", "TABLE2_ROW4_BCOMMENT", "TABLE2_ROW2_STR", "UTF8"])
def test_framed_sets(name, reserved):
    """Framing at the producer (Section 7.1): the reserved byte leaves every pattern and
    becomes a kind of its own, on both sides."""
    defs = T.as_tuples(SETS[name])
    lx = P.Lexer.compile_framed(defs, reserved)
    assert lx.info()["nkinds"] == len(defs) + 1
    _agree(lx, oracle.OracleSet(defs, reserved=reserved).cert(), (name, reserved))


def test_framed_random_sets():
    for seed in range(150):
        defs = rand_set(seed, "abc")
        for r in (ord("a"), ord(";")):
            _agree(P.Lexer.compile_framed(defs, r), oracle.OracleSet(defs, reserved=r).cert(), (defs, r))


def test_random_sets():
    for seed in range(400):
        defs = rand_set(seed, "abc")
        _agree(P.Lexer.compile(defs), oracle.OracleSet(defs).cert(), defs)
    for seed in range(1000, 1200):
        defs = rand_set(seed, "abcd")
        _agree(P.Lexer.compile(defs), oracle.OracleSet(defs).cert(), defs)


def _rand_table(rng: random.Random):
    n = rng.randint(1, 7)
    nxt = np.full((n, 256), -1, np.int32)
    alpha = [ord(c) for c in "abc;"]
    for q in range(n):
        for b in alpha:
            if rng.random() < 0.45:
                nxt[q, b] = rng.randrange(n)
    acc = [rng.choice([-1, -1, 0, 1, 2]) for _ in range(n)]
    disc = [rng.random() < 0.5 for _ in range(3)]
    return nxt, acc, rng.randrange(n), disc


def test_random_hand_built_tables():
    """Arbitrary tables with unreachable and dead states (Section 4.1's two halves of Q+)."""
    rng = random.Random(5)
    for _ in range(500):
        nxt, acc, q0, disc = _rand_table(rng)
        _agree(P.Lexer.from_table(nxt, acc, q0, disc), oracle.cert_table(nxt, acc, q0, disc), (nxt, acc, q0))


def test_paper_tables():
    t = np.full((4, 256), -1, np.int32)
    t[0, ord("a")] = 2
    t[2, ord("b")] = 1
    t[0, ord("b")] = 3
    lx = P.Lexer.from_table(t, [-1, -1, -1, 1], 0, [0, 0])
    assert lx.cert() == {ord("b")} and ord("a") in lx.cert(raw=True)


def test_syntax_errors_are_reported():
    for bad in ["(", "a)", "[", "[z-a]", "*a", "a{2", "a{3,1}", "\\q", "[^\\x00-\\xff]"]:
        with pytest.raises(P.LexError) as ei:
            P.Lexer.compile([(bad, 0, False)])
        assert ei.value.code == P.LEX_ESYNTAX, bad
        with pytest.raises(ValueError):
            oracle.OracleSet([(bad, 0, False)])


def test_kind_limit():
    with pytest.raises(P.LexError) as ei:
        P.Lexer.compile([("a", 0, False)] * 256)
    assert ei.value.code == P.LEX_ELIMIT
