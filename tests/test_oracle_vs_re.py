"""The oracle's NFA lexer against an independent tokenizer built on Python's ``re`` engine
(special case reducing to a library routine), on tiny random inputs.  CPU only."""
import random

import oracle
import pyref
from workloads import tokensets as T

from randsets import rand_set


def _compare(defs, alphabet: bytes, trials: int, maxlen: int, seed: int):
    s = oracle.OracleSet(defs)
    ref = pyref.compile_defs(defs)
    rng = random.Random(seed)
    for _ in range(trials):
        n = rng.randint(0, maxlen)
        w = bytes(rng.choice(alphabet) for _ in range(n))
        k, l, con = s.lex(w)
        rt, rcon = pyref.lex(ref, w)
        assert con == rcon, (defs, w)
        assert list(zip(k.tolist(), l.tolist())) == rt, (defs, w)


def test_random_sets_vs_re():
    for seed in range(300):
        _compare(rand_set(seed, "abc"), b"abc", 40, 10, seed)


def test_named_sets_vs_re():
    cases = [
        (T.CLIKE_L, b'ab1 \t\n/*"\\=!&|<>+-.;x'),
        (T.CLIKE_D, b'ab1 \n/"\\=&'),
        (T.CLIKE_B, b"a/* \n1"),
        (T.JSON, b'"\\u0aF1-.eE+ \ntrufalsn{}[]:,'),
        (T.UTF8, bytes([0x41, 0xC3, 0xA9, 0xE2, 0x82, 0xAC, 0xF0, 0x9F, 0x98, 0x80, 0xFF, 0xC0])),
    ]
    for i, (defs, alpha) in enumerate(cases):
        _compare(T.as_tuples(defs), alpha, 600, 14, 1000 + i)


def test_priority_ties_vs_re():
    defs = [("[a-c]+", 1, False), ("ab|ba", 0, False), ("a(b|c)", 0, False), ("c+", 2, True)]
    _compare(defs, b"abc", 500, 10, 7)
