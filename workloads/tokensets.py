"""Token-set transcriptions used as inputs by both the library and the oracle.

Patterns are in the byte-regex dialect both sides parse independently: literals, ``.``,
classes ``[..]``/``[^..]`` with ranges, groups, ``|``, postfix ``* + ? {m} {m,} {m,n}``,
escapes ``\\n \\t \\r \\f \\v \\0 \\xHH`` and a backslash before any non-alphanumeric byte.
Languages are over bytes.  Kind ids follow declaration order; every priority is 0 unless
stated (no same-length ties arise in these sets).  ``discard`` marks membership of the
discarded set I of Section 5.

The C-like, JSON and log-line sets transcribe the workloads the paper measures and the
rows of its applicability table (Section 7, Table 2); ``Expected`` records the useful
certified sets the paper prints for them, where it prints one.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class TokDef:
    name: str
    pattern: str
    priority: int = 0
    discard: bool = False

    def as_tuple(self):
        return (self.pattern, self.priority, self.discard)


def _defs(*rows):
    return tuple(TokDef(*r) for r in rows)


IDENT = ("IDENT", r"[A-Za-z_][A-Za-z0-9_]*")
INT = ("INT", r"[0-9]+")
# 24 operator spellings; a lone '&' or '|' is not a token.
OP = ("OP", r"\+|-|\*|/|%|=|==|!=|<|<=|>|>=|&&|\|\||!|\(|\)|\{|\}|\[|\]|;|,|\.")
OP_SPELLINGS = ("+", "-", "*", "/", "%", "=", "==", "!=", "<", "<=", ">", ">=", "&&", "||",
                "!", "(", ")", "{", "}", "[", "]", ";", ",", ".")
# String literal: no raw newline, backslash escapes any non-newline byte.
STR = ("STR", r'"([^"\\\n]|\\[^\n])*"')
LCOMMENT = ("LCOMMENT", r"//[^\n]*")
# Block comment in its C form: ends at the first "*/", does not nest.
BCOMMENT = ("BCOMMENT", r"/\*([^*]|\*+[^*/])*\*+/")

# Split-friendly C-like set: newline is its own token, spaces and tabs a separate run.
CLIKE_L = _defs(IDENT, INT, OP, STR, ("SPACE", r"[ \t]+"), ("NEWLINE", r"\n"), LCOMMENT)

# Conventional C-like set: one whitespace run including newline; whitespace and line
# comments discarded.
CLIKE_D = _defs(IDENT, INT, OP, STR, ("SPACE", r"[ \t\n]+", 0, True), LCOMMENT + (0, True))

# CLIKE_D plus unrestricted block comments (discarded).
CLIKE_B = CLIKE_D + _defs(BCOMMENT + (0, True))

JSON = _defs(
    ("STRING", r'"([^"\\\x00-\x1F]|\\["\\/bfnrt]|\\u[0-9A-Fa-f]{4})*"'),
    ("NUMBER", r"-?(0|[1-9][0-9]*)(\.[0-9]+)?([eE][+-]?[0-9]+)?"),
    ("TRUE", r"true"),
    ("FALSE", r"false"),
    ("NULL", r"null"),
    ("PUNCT", r"[{}\[\]:,]"),
    ("WS", r"[ \t\n\r]+", 0, True),
)

LOG = _defs(("LINE", r"[^\n]+"), ("NL", r"\n"))

# Applicability-table rows (Table 2) in our own transcription.
ROW1_OPS = "+-*/%=<>!&|^~?:;,.(){}[]"  # 24 single-byte operators and punctuation
_ROW1_OP = ("OP", "[" + "".join("\\" + c for c in ROW1_OPS) + "]")
TABLE2_ROW1 = _defs(IDENT, ("NUMBER", r"[0-9]+"), ("WS", r"[ \t\n]+", 0, True), _ROW1_OP)
TABLE2_ROW2_STR = TABLE2_ROW1 + _defs(STR)
TABLE2_ROW3_LCOMMENT = TABLE2_ROW1 + _defs(LCOMMENT + (0, True))
TABLE2_ROW4_BCOMMENT = TABLE2_ROW1 + _defs(BCOMMENT + (0, True))
# Split-friendly base with every body barred from the bytes that open another string
# or comment ('"' and '/').
TABLE2_BARRED = _defs(
    IDENT, INT, OP,
    ("STR", r'"([^"\\\n/]|\\[^\n/])*"'),
    ("SPACE", r"[ \t]+", 0, True), ("NEWLINE", r"\n"),
    ("LCOMMENT", r'//[^\n"/]*', 0, True),
    ("BCOMMENT", r'/\*([^*"/]|\*+[^*/"])*\*+/', 0, True),
)
# Split-friendly base with ordinary bodies, the block comment barred from crossing a line.
TABLE2_LINE_BLOCK = _defs(
    IDENT, INT, OP, STR, ("SPACE", r"[ \t]+", 0, True), ("NEWLINE", r"\n"),
    LCOMMENT + (0, True),
    ("BCOMMENT", r"/\*([^*\n]|\*+[^*/\n])*\*+/", 0, True),
)
# Split-friendly set with comments and whitespace discarded (right column of Table 2).
CLIKE_L_I = _defs(IDENT, INT, OP, STR, ("SPACE", r"[ \t]+", 0, True), ("NEWLINE", r"\n"),
                  LCOMMENT + (0, True))
CLIKE_L_BLOCK_I = CLIKE_L_I + _defs(BCOMMENT + (0, True))

# UTF-8 encoding forms, one kind per form length, plain lead/continuation classes.
UTF8 = _defs(
    ("U1", r"[\x00-\x7F]"),
    ("U2", r"[\xC2-\xDF][\x80-\xBF]"),
    ("U3", r"[\xE0-\xEF][\x80-\xBF]{2}"),
    ("U4", r"[\xF0-\xF4][\x80-\xBF]{3}"),
)

NAMED = {
    "clike_l": CLIKE_L, "clike_d": CLIKE_D, "clike_b": CLIKE_B, "json": JSON, "log": LOG,
}

NL = {0x0A}
# Useful certified sets the paper prints or the configs state: (exact, modulo I).
EXPECTED = {
    "clike_l": (NL, NL),
    "clike_d": (set(), NL),
    "clike_b": (set(), set()),
    "json": (set(), {0x09, 0x0A, 0x0D}),
    "log": (NL, NL),
}


def as_tuples(defs):
    return [d.as_tuple() for d in defs]


def kind_names(defs):
    return [d.name for d in defs]


def discard_kinds(defs):
    return frozenset(i for i, d in enumerate(defs) if d.discard)
