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
