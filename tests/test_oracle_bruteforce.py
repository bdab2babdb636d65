"""Exhaustive checks of the oracle over every short string (CPU only).

For each token set and every string up to the length bound over a small alphabet the
oracle's own sweep (orc_bruteforce) asserts:
  * Lemma 1 / Lemma 3 -- every certified occurrence before con(w) is a token boundary;
  * Theorem 1 / Corollary 1 -- splitting at every useful exact occurrence, and at each one
    alone, reproduces the serial stream (and, on malformed input, its prefix and halt);
  * Theorem 3 and the malformed-input reading -- the same modulo I after pi_I;
  * Proposition 3 -- exact certificates are certified modulo I;
  * Theorem 2 -- each consumed, rejected byte has a witness lexing as one token, and when
    that witness fits the bound the enumeration saw the byte strictly inside a token.
These tie the certificate checker (its own automaton) to the NFA lexer: a certificate that
admits too much breaks the split comparisons, one that refuses too much fails the witness.
"""
import pytest

import oracle
from workloads import tokensets as T

from randsets import rand_set

VIOLATIONS = ("lemma1_viol", "thm1_viol", "cor1_viol", "thm3_viol", "malformed_i_viol",
              "prop3_viol", "witness_viol", "necessity_viol")


def _check(st):
    bad = {k: st[k] for k in VIOLATIONS if st[k]}
    assert not bad, bad


def test_random_sets_three_symbols_len8():
    """400 seeded random token sets over {a,b,c}, every string of length 1..8."""
    tot = {"admitted": 0, "refused_safe": 0, "consumed": 0, "splits": 0}
    for seed in range(400):
        defs = rand_set(seed, "abc")
        s = oracle.OracleSet(defs)
        st = s.bruteforce(b"abc", 8)
        assert st["strings"] == 9840
        _check(st)
        # Section 5: with I empty the two conditions coincide
        c0 = oracle.OracleSet([(p, pr, False) for p, pr, _ in defs]).cert()
        assert c0["discard_raw"] == c0["exact_raw"]
        tot["admitted"] += st["pairs_admitted_i"]
        tot["refused_safe"] += st["pairs_refused_safe"]
        tot["consumed"] += st["pairs_consumed"]
        tot["splits"] += st["mode_splits"]
    # the sweep must actually exercise both conditions
    assert tot["admitted"] > 50 and tot["splits"] > 100000
    print("sweep totals", tot)


def test_random_sets_four_symbols_len6():
    """The independently parameterised four-symbol variant, to a shorter bound."""
    for seed in range(1000, 1150):
        s = oracle.OracleSet(rand_set(seed, "abcd"))
        _check(s.bruteforce(b"abcd", 6))


PROJECTED = [
    ("clike_l", T.CLIKE_L, b'a/" \n'),
    ("clike_l_ops", T.CLIKE_L, b"1=!&\n"),
    ("clike_d", T.CLIKE_D, b'a/\n "'),
    ("clike_b", T.CLIKE_B, b"/*a\n "),
    ("json_str", T.JSON, b'"\\1\n '),
    ("json_num", T.JSON, b"1.e-\n"),
    ("json_kw", T.JSON, b"true\n"),
    ("log", T.LOG, b"ab\n"),
    ("utf8", T.UTF8, b"a\xc3\xa9\xe2\x80"),
]


@pytest.mark.parametrize("name,defs,alpha", PROJECTED, ids=[p[0] for p in PROJECTED])
def test_projected_config_sets(name, defs, alpha):
    """The configs' token sets restricted to small alphabets, every string up to length 7."""
    s = oracle.OracleSet(T.as_tuples(defs))
    st = s.bruteforce(alpha, 7)
    _check(st)
    assert st["strings"] == sum(len(alpha) ** k for k in range(1, 8))


@pytest.mark.slow
@pytest.mark.parametrize("name,defs,alpha", PROJECTED[:4], ids=[p[0] for p in PROJECTED[:4]])
def test_projected_config_sets_len8(name, defs, alpha):
    s = oracle.OracleSet(T.as_tuples(defs))
    _check(s.bruteforce(alpha, 8))
