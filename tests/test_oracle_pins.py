"""Pins of the oracle against what the paper fixes (printed examples, printed table cells,
closed forms, special cases).  CPU only.

Each test names the passage it restates.  Together they are chosen so that a plausible
slip in the oracle -- a dropped clause of Definition 2 or 3, delta instead of delta+, a
missing useful-set filter, a wrong tie-break, an off-by-one in longest match, a wrong
truncation rule -- fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

NL = 0x0A


def oset(defs):
    return oracle.OracleSet(T.as_tuples(defs) if defs and isinstance(defs[0], T.TokDef) else defs)


def load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def ranges(rs):
    return {b for lo, hi in rs for b in range(lo, hi + 1)}


# ----------------------------------------------------------------- Figure 2
def test_fig2_tokens_and_split(golden_dir):
    g = load(golden_dir, "fig2_split_example.json")
    s = oset(T.CLIKE_L)
    names = T.kind_names(T.CLIKE_L)
    w = g["input"].encode()
    kinds, lens, con = s.lex(w)
    assert con == len(w)
    ext, off = [], 0
    for l in lens:
        ext.append([off, off + int(l) - 1])
        off += int(l)
    assert ext == g["extents"]
    assert [names[k] for k in kinds] == g["kinds"]
    assert w[g["certified_offset"]] in s.cert()["exact"]
    ck, cl, err = s.lex_chunked(w, [c[0] for c in g["chunks"][1:]])
    assert err == len(w)
    assert list(ck) == list(kinds) and list(cl) == list(lens)


# ------------------------------------------------------- Table 2 and configs
def test_table2_rows(golden_dir):
    g = load(golden_dir, "table2_applicability.json")
    ops = {ord(c) for c in T.ROW1_OPS}
    assert len(ops) == 24

    def expand(v):
        if v == "ops24":
            return ops
        if v == "ops24+[9,10,32]":
            return ops | {9, 10, 32}
        return set(v)

    for row in g["rows"]:
        c = oset(getattr(T, row["set"])).cert()
        assert set(c["exact"]) == expand(row["exact"]), row["row"]
        assert set(c["discard"]) == expand(row["modulo"]), row["row"]


@pytest.mark.parametrize("name", sorted(T.NAMED))
def test_config_token_sets(name):
    c = oset(T.NAMED[name]).cert()
    ex, mo = T.EXPECTED[name]
    assert set(c["exact"]) == ex
    assert set(c["discard"]) == mo
    # Proposition 3: exact certificates survive modulo any I
    assert c["exact_raw"] <= c["discard_raw"]


def _without_discard(defs):
    return [(d.pattern, d.priority, False) for d in defs]


@pytest.mark.parametrize("name", sorted(T.NAMED) + ["TABLE2_ROW1", "TABLE2_ROW2_STR",
                                                     "TABLE2_ROW3_LCOMMENT", "TABLE2_ROW4_BCOMMENT",
                                                     "CLIKE_L_BLOCK_I", "TABLE2_BARRED", "UTF8"])
def test_empty_discard_set_recovers_exact(name):
    """Section 5: with I empty, Definition 3 reduces to Definition 2."""
    defs = T.NAMED.get(name) or getattr(T, name)
    c = oracle.OracleSet(_without_discard(defs)).cert()
    assert c["discard_raw"] == c["exact_raw"]
    assert c["discard"] == c["exact"]


# ---------------------------------------------------------------- UTF-8
def test_utf8_instance(golden_dir):
    g = load(golden_dir, "utf8_certified.json")
    c = oset(T.UTF8).cert()
    assert set(c["exact"]) == ranges(g["useful_ranges"])
    assert not (set(c["exact_raw"]) & ranges(g["not_certified_ranges"]))
    vac = ranges(g["vacuous_ranges"])
    assert vac <= set(c["exact_raw"])          # certified (vacuously, Proposition 1)
    assert not (vac & set(c["exact"]))          # withheld (Corollary 2)
    assert not (vac & set(c["consumed"]))


# ----------------------------------------------------- counterexamples
def _case(golden_dir, cid):
    for c in load(golden_dir, "counterexamples.json")["cases"]:
        if c["id"] == cid:
            return c
    raise KeyError(cid)


def test_nullable_reentry(golden_dir):
    c = _case(golden_dir, "nullable_reentry")
    s = oracle.OracleSet(c["defs"])
    ci = s.cert()
    assert ci["reentrant"] and c["byte"] not in ci["exact_raw"]
    k, l, con = s.lex(b"aa")
    assert list(l) == [2] and con == 2
    ck, cl, err = s.lex_chunked(b"aa", [1])
    assert len(ck) == c["split_at_1_tokens"]  # the naive certificate would be wrong
    # positive-length tokens: an accepting q0 never emits the empty word
    k, l, con = s.lex(b"b")
    assert len(k) == 0 and con == 0


def test_cyclic_reentry(golden_dir):
    c = _case(golden_dir, "cyclic_reentry")
    s = oracle.OracleSet(c["defs"])
    ci = s.cert()
    assert ci["reentrant"] and c["byte"] not in ci["exact_raw"]
    k, l, con = s.lex(b"abc")
    assert list(l) == [3] and con == 3


def test_fig1a_semicolon(golden_dir):
    c = _case(golden_dir, "fig1a")
    ci = oracle.OracleSet(c["defs"]).cert()
    assert not ci["reentrant"]
    assert ci["exact"] == {c["byte"]}


def test_strict_extension(golden_dir):
    """Proposition 3's example: newline uncertified exactly, certified modulo I."""
    c = _case(golden_dir, "strict_extension")
    ci = oracle.OracleSet(c["defs"]).cert()
    assert c["byte"] not in ci["exact"] and c["byte"] in ci["discard"]


def test_conservative_witness(golden_dir):
    """Section 6.1: b is refused modulo I (clause 2 fails) yet every split at b is safe."""
    c = _case(golden_dir, "conservative_witness")
    s = oracle.OracleSet(c["defs"])
    assert c["byte"] not in s.cert()["discard_raw"]
    st = s.bruteforce(b"abc", 8)
    assert st["pairs_refused_safe"] >= 1
    assert st["thm3_viol"] == 0 and st["thm1_viol"] == 0


def test_quadratic_lookahead(golden_dir):
    """Section 9: ';' certifies but never occurs in a^N, so one chunk; N tokens (a, 1)."""
    c = _case(golden_dir, "quadratic_lookahead")
    s = oracle.OracleSet(c["defs"])
    assert s.cert()["exact"] == {c["byte"]}
    n = 1500
    k, l, con = s.lex(b"a" * n)
    assert con == n and len(k) == n and set(l.tolist()) == {1} and set(k.tolist()) == {0}


def test_clause1_accepting_state_required():
    """Definition 3 clause 1: a cut inside a non-accepting state cannot end the left chunk on a
    complete token.  One discarded kind ab|b: q_a consumes b into the state q0 reaches on b."""
    s = oracle.OracleSet([("ab|b", 0, True)])
    ci = s.cert()
    assert ord("b") not in ci["discard_raw"]
    _, _, err = s.lex_chunked(b"ab", [1], discard=True)
    assert err == 0  # the left slice "a" does not tokenize: the cut would be unsound


def test_clause3_kept_token_blocks():
    """Definition 3 clause 3: a run of a kept kind must not be severed."""
    s = oracle.OracleSet([("a+", 0, False), ("b", 0, True)])
    assert ord("a") not in s.cert()["discard_raw"]
    k, _, _ = s.lex_chunked(b"aa", [1], discard=True)
    assert len(k) == 2  # serial gives one kept token


def test_tie_break_priority_then_index():
    """Section 3: same-length ties go to the lower priority number, then the lower index."""
    s = oracle.OracleSet([("[a-z]+", 1, False), ("if", 0, False)])
    k, l, _ = s.lex(b"if")
    assert list(k) == [1] and list(l) == [2]
    k, l, _ = s.lex(b"iff")
    assert list(k) == [0] and list(l) == [3]
    s = oracle.OracleSet([("if", 0, False), ("[a-z]+", 0, False)])
    assert list(s.lex(b"if")[0]) == [0]
    s = oracle.OracleSet([("[a-z]+", 0, False), ("if", 0, False)])
    assert list(s.lex(b"if")[0]) == [0]


# --------------------------------------------------- hand-built automata
def _table(n):
    return np.full((n, 256), -1, np.int32)


def test_empty_language_chain():
    """Section 4.1: T1 = ab.empty beside T2 = b.  q0 -a-> q2 -b-> q1 (dead), q0 -b-> q3."""
    t = _table(4)
    t[0, ord("a")] = 2
    t[2, ord("b")] = 1
    t[0, ord("b")] = 3
    acc = [-1, -1, -1, 1]
    c = oracle.cert_table(t, acc, q0=0, discard=[0, 0])
    assert ord("b") in c["exact"]                 # over delta+ the chain is invisible
    assert ord("a") in c["exact_raw"] and ord("a") not in c["exact"]  # vacuous
    assert c["nstates"] == 2


def test_detached_state():
    """Section 4.1: T2 = b plus a detached q4 -b-> q5 accepting; b stays certified.
    (q4 is given a label of its own so that minimisation cannot fold it into q0.)"""
    t = _table(6)
    t[0, ord("b")] = 3
    t[4, ord("b")] = 5
    acc = [-1, -1, -1, 1, 0, 1]
    c = oracle.cert_table(t, acc, q0=0, discard=[0, 0])
    assert c["exact"] == {ord("b")}
    assert c["nstates"] == 2


def test_empty_token_set_table():
    """q0 not live: nothing is useful."""
    t = _table(2)
    t[0, ord("a")] = 1
    c = oracle.cert_table(t, [-1, -1], q0=0, discard=[0])
    assert not c["q0_live_state"] and not c["exact"] and not c["discard"]


# ---------------------------------------------------------- Section 5, 7
def test_line_comment_cut_reveals_kept_token():
    """Section 5: cutting //ab between a and b leaves //a (discarded) and b (kept)."""
    s = oset(T.CLIKE_D)
    assert ord("b") not in s.cert()["discard"]
    k, l, err = s.lex_chunked(b"//ab", [3], discard=True)
    assert err == 4 and list(k) == [0] and list(l) == [1]  # IDENT b survives pi_I
    k, l, con = s.lex(b"//ab", discard=True)
    assert len(k) == 0 and con == 4


def test_block_comment_split_relexes():
    """Section 7: a block comment severed at a newline re-lexes as six kept tokens."""
    s = oset(T.CLIKE_B)
    w = b"/* a\nb */"
    k, _, con = s.lex(w, discard=True)
    assert con == len(w) and len(k) == 0
    k, _, err = s.lex_chunked(w, [4], discard=True)
    assert err == len(w) and len(k) == 6


def test_witnesses_are_single_tokens():
    """Theorem 2: every consumed, uncertified byte has a witness u b v lexing as one token."""
    for defs in (T.CLIKE_L, T.CLIKE_D, T.JSON, T.UTF8, T.TABLE2_ROW1):
        s = oset(defs)
        c = s.cert()
        checked = 0
        for b in sorted(c["consumed"] - c["exact_raw"]):
            w, boff = s.witness(b)
            assert w[boff] == b and boff >= 1
            k, l, con = s.lex(w)
            assert con == len(w) and len(k) == 1, (b, w)
            checked += 1
        for b in c["exact_raw"]:
            assert s.witness(b) is None
        assert checked > 0 or defs is T.TABLE2_ROW1


# ------------------------------------------------------ Section 8.2 pin
def test_planning_workload_token_count(golden_dir):
    g = load(golden_dir, "planning_workload.json")
    s = oset(T.LOG)
    w = workloads.loglines(g["n"], g["period"])
    k, l, con = s.lex(w)
    assert con == g["n"] and len(k) == g["tokens_with_newlines"]
    assert int(l.astype(np.uint64).sum()) == g["n"]
    w = workloads.loglines(g["n"], None)
    k, l, con = s.lex(w)
    assert con == g["n"] and len(k) == g["tokens_without_newline"]


# -------------------------------------------- malformed input (Corollary 1)
def test_malformed_prefix_rule():
    s = oset(T.CLIKE_L)
    w = b"a = 1;\nb = 2 & 3;\nc = 4;\n"
    k, l, con = s.lex(w)
    assert con == w.index(b"&")
    cuts = [i for i, c in enumerate(w) if c == NL and i > 0]
    ck, cl, err = s.lex_chunked(w, cuts)
    assert err == con and list(ck) == list(k) and list(cl) == list(l)
