"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of oracle.cc (a dropped clause of
Definition 2 or 3, delta instead of delta+, a missing useful-set filter, a reversed
tie-break, an off-by-one in longest match, a missing truncation, a mis-seeded closure),
builds it into a temporary library and runs the pin suite against it (the framing pins for
the framing mutants): every mutant must fail at least one pin.  The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "no_reentrancy": ("bool A = (q == q0) && !reent;", "bool A = (q == q0);"),
    "reentrancy_self_loop_only": ("if (dp(q, b) == q0) reent = true;",
                                  "if (dp(q, b) == q0 && q == q0) reent = true;"),
    "no_clause1": ("bool C = d.acc[q] >= 0 && t0 >= 0", "bool C = t0 >= 0"),
    "no_clause2": ("t0 >= 0 && t0 == t && !reaches_kept[q]", "t0 >= 0 && !reaches_kept[q]"),
    "no_clause3": ("t0 == t && !reaches_kept[q];", "t0 == t;"),
    "kept_seed_inverted": ("if (d.acc[q] >= 0 && !discard[d.acc[q]]) {",
                           "if (d.acc[q] >= 0 && discard[d.acc[q]]) {"),
    "no_useful_filter": ("if (exact && t0 >= 0) setbit(out->exact_useful, b);",
                         "if (exact) setbit(out->exact_useful, b);"),
    "no_useful_filter_modulo": ("if (modi && t0 >= 0) setbit(out->discard_useful, b);",
                                "if (modi) setbit(out->discard_useful, b);"),
    "trim_without_coaccessible": ("live[q] = reach[q] && coacc[q];", "live[q] = reach[q];"),
    "trim_without_reachable": ("live[q] = reach[q] && coacc[q];", "live[q] = coacc[q];"),
    "tie_index_reversed": ("(S->prio[k] == S->prio[best] && k < best)",
                           "(S->prio[k] == S->prio[best] && k > best)"),
    "tie_priority_reversed": ("(l == best_len && (S->prio[k] < S->prio[best] ||",
                              "(l == best_len && (S->prio[k] > S->prio[best] ||"),
    "length_off_by_one": ("best = j + 1 - i;", "best = j - i;"),
    "first_not_longest": ("best = j + 1 - i;\n        break;", "best = j + 1 - i;\n        return best;"),
    "no_truncation": ("if (con < hi - lo) return lo + con;", "(void)con;"),
    # framing at the producer (Section 7.1), held by the framing pins
    "framing_no_exclusion": ("if (nd.kind == N_SET) nd.set.w[r >> 6] &= ~((uint64_t)1 << (r & 63));",
                             "(void)nd;", "test_framing.py"),
    "framing_discard_inverted": ("S->discard.push_back(r_discard ? 1 : 0);",
                                 "S->discard.push_back(r_discard ? 0 : 1);", "test_framing.py"),
    "framing_wrong_byte": ("ast[0].set.add((int)r);", "ast[0].set.add((int)r + 1);", "test_framing.py"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "oracle.cc")).read()
    a, b, *target = MUTANTS[name]
    target = target[0] if target else "test_oracle_pins.py"
    assert a in src, f"mutation site vanished: {name}"
    m = tmp_path / "mutant.cc"
    m.write_text(src.replace(a, b, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "oracle"),
                    "-o", str(lib), str(m)], check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", target)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
