"""Applicability of certified splitting to a token set: which bytes certify a cut, exactly
(Definition 2) and modulo the declared discarded kinds I (Definition 3), with the useful
subsets the planner cuts at (Corollary 2, Proposition 2), and what a scan of each mode
therefore does on the GPU.

    python -m paper_2608_03473_amd.applicability               # the Table 2 transcriptions
    python -m paper_2608_03473_amd.applicability SET.json      # a token set of one's own
    python -m paper_2608_03473_amd.applicability --json ...    # machine-readable
    python -m paper_2608_03473_amd.applicability --reserve 0x1E  # each set framed by a byte

A token-set file is a JSON list of objects {"name", "pattern", "priority" (default 0),
"discard" (default false)}; patterns use the library's byte regex dialect.  The sets are
computed by the library's compiler (lex_cert), the same one every scan uses.  With
--reserve r every set is first framed by the byte r (Section 7.1: r leaves every pattern
and becomes a token of its own, lex_compile_framed).
"""
from __future__ import annotations

import argparse
import json
import sys

from . import abi
from .lexer import Lexer

# The rows of Table 2 as transcribed in workloads/tokensets.py: (set name, what it is).
TABLE2 = [
    ("TABLE2_ROW1", "identifiers, numbers, whitespace runs, 24 single-byte operators"),
    ("TABLE2_ROW2_STR", "row 1 plus string literals without raw newlines"),
    ("TABLE2_ROW3_LCOMMENT", "row 1 plus // line comments"),
    ("TABLE2_ROW4_BCOMMENT", "row 1 plus block comments"),
    ("JSON", "JSON lexical forms over bytes"),
    ("LOG", "log lines: non-newline runs and newline"),
    ("CLIKE_D", "C-like, whitespace runs that include newline"),
    ("CLIKE_L_I", "C-like, newline a token of its own"),
    ("CLIKE_L_BLOCK_I", "newline its own token, plus block comments"),
    ("TABLE2_BARRED", "three kinds, each body barred from the bytes that open another"),
    ("TABLE2_LINE_BLOCK", "block comments barred from crossing a line"),
]


def show_bytes(bs) -> str:
    """A byte set as ranges of printable characters and hex escapes."""
    bs = sorted(bs)
    if not bs:
        return "(none)"
    parts, i = [], 0
    while i < len(bs):
        j = i
        while j + 1 < len(bs) and bs[j + 1] == bs[j] + 1:
            j += 1
        one = lambda b: chr(b) if 0x21 <= b <= 0x7E else f"\\x{b:02X}"  # noqa: E731
        parts.append(one(bs[i]) if i == j else f"{one(bs[i])}-{one(bs[j])}" if j > i + 1 else f"{one(bs[i])} {one(bs[j])}")
        i = j + 1
    return " ".join(parts)


def analyse(defs, reserve: int | None = None) -> dict:
    """Certified and useful sets of both modes, and the scan each mode gets."""
    lx = Lexer.compile(defs) if reserve is None else Lexer.compile_framed(defs, reserve)
    info = lx.info()
    out = {"kinds": info["nkinds"], "rows": info["nrows"], "monotone": bool(info["monotone"])}
    for mode, key in ((abi.LEX_MODE_EXACT, "exact"), (abi.LEX_MODE_DISCARD, "discard")):
        raw, useful = lx.cert(mode, raw=True), lx.cert(mode)
        plan = lx.plan(1 << 20, mode)  # a 1 MiB scan of this mode
        if useful:
            how = "splits at its useful certified bytes"
        elif plan["hybrid"]:
            how = "refused: no useful certified byte; the hybrid plan splits it speculatively"
        else:
            how = "one slice"
        out[key] = {"certified": sorted(raw), "useful": sorted(useful), "scan": how,
                    "windowed_emit": bool(plan["windowed"])}
    return out


def _load(path):
    with open(path, encoding="utf-8") as f:
        defs = json.load(f)
    if not isinstance(defs, list) or not defs:
        raise ValueError("a token-set file holds a non-empty JSON list of token definitions")
    for d in defs:
        if not isinstance(d, dict) or "pattern" not in d:
            raise ValueError("each definition needs at least a 'pattern'")
    return defs


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("files", nargs="*", help="token-set JSON files (default: the Table 2 transcriptions)")
    ap.add_argument("--json", action="store_true", help="one JSON object per token set")
    ap.add_argument("--reserve", type=lambda v: int(v, 0), default=None,
                    help="frame every set by this byte (e.g. 0x1E) before analysing it")
    args = ap.parse_args(argv)
    if args.reserve is not None and not 0 <= args.reserve <= 255:
        ap.error("--reserve takes a byte value 0..255")
    if args.files:
        sets = [(f, None, _load(f)) for f in args.files]
    else:
        from workloads import tokensets as T

        sets = [(name, what, [d.as_tuple() for d in getattr(T, name)]) for name, what in TABLE2]
    for name, what, defs in sets:
        r = analyse(defs, args.reserve)
        if args.reserve is not None:
            name = f"{name} framed by {show_bytes([args.reserve])}"
        if args.json:
            print(json.dumps({"set": name, **({"about": what} if what else {}), **r}))
            continue
        print(f"{name}" + (f" — {what}" if what else ""))
        print(f"  {r['kinds']} kinds, {r['rows']} table rows, {'monotone' if r['monotone'] else 'not monotone'}")
        for key, label in (("exact", "exact (E, E_u)"), ("discard", "modulo I (D, D_u)")):
            m = r[key]
            print(f"  {label:18s} certified {show_bytes(m['certified'])}")
            print(f"  {'':18s} useful    {show_bytes(m['useful'])}   -> {m['scan']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
