"""An independent longest-match tokenizer built on Python's own regex engine.

Used only to pin the oracle's lexer on tiny inputs: for every offset and every kind it asks
``re.fullmatch`` for each candidate length and keeps the longest positive one, breaking a
same-length tie by (priority, kind index) as Section 3 states.  It shares nothing with the
oracle's NFA code.
"""
import re


def compile_defs(defs):
    out = []
    for pat, prio, disc in defs:
        if isinstance(pat, str):
            pat = pat.encode("latin-1")
        out.append((re.compile(pat, re.DOTALL), prio, disc))
    return out


def lex(cdefs, w: bytes):
    i, n, toks = 0, len(w), []
    while i < n:
        best = None  # (len, -prio, -k) maximised
        for k, (rx, prio, _) in enumerate(cdefs):
            for l in range(n - i, 0, -1):
                if rx.fullmatch(w, i, i + l):
                    cand = (l, -prio, -k)
                    if best is None or cand > best:
                        best = cand
                    break
        if best is None:
            break
        toks.append((-best[2], best[0]))
        i += best[0]
    return toks, i


def lex_framed(cdefs, w: bytes, r: int):
    """The set framed by the reserved byte r (Section 7.1), from the languages themselves:
    kind k keeps exactly its words that do not contain r, and kind len(cdefs) is the
    one-byte word r (priority 0)."""
    i, n, toks = 0, len(w), []
    rb = bytes([r])
    while i < n:
        best = None
        for k, (rx, prio, _) in enumerate(cdefs):
            for l in range(n - i, 0, -1):
                if rb not in w[i:i + l] and rx.fullmatch(w, i, i + l):
                    cand = (l, -prio, -k)
                    if best is None or cand > best:
                        best = cand
                    break
        if w[i] == r:
            cand = (1, 0, -len(cdefs))
            if best is None or cand > best:
                best = cand
        if best is None:
            break
        toks.append((-best[2], best[0]))
        i += best[0]
    return toks, i
