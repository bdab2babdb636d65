"""A slow host model of the GPU lane walker, run on the library's packed tables.

It restates, in plain Python, what one lane does with the packed table of include/lex.h's
library (entry bits: COUNT 0, EMIT 1, row swizzle (row & 31) in 2..6, ACC 7, next-row byte
offset (row * 1024) in 10..23, kind in 24..31; row r keeps byte b's entry at index
r * 256 + (b ^ (r & 31)); row 0 = token start, SINK after the DFA rows, FAIL after SINK for
non-monotone automata).
Tests use it to check the *tables* against the oracle on the CPU before any kernel runs.
"""
ROWMASK, ACC, EMIT, COUNT = 0x00FFFC00, 1 << 7, 1 << 1, 1 << 0
INFO_ACC, INFO_COUNT = 0x80, 0x40


class Model:
    def __init__(self, lexer, mode):
        self.T, self.info, self.kind = lexer.tables(mode & 1)
        inf = lexer.info()
        # row states are kept as row index * 256, the index of the row's first entry
        self.sink = (1 + inf["nstates"]) * 256
        self.mono = bool(inf["monotone"])
        self.fail = self.sink if self.mono else (2 + inf["nstates"]) * 256

    def walk(self, w: bytes, s: int, e: int):
        """Tokens (kind, length, start) written by a lane on [s, e), and its halt offset or None."""
        T, out = self.T, []
        st, tok, lacc, lrow = 0, s, s, 0

        def recover(upto):  # non-monotone automata only (FAIL != SINK)
            nonlocal st, tok, lacc, lrow
            while st == self.fail:
                if lacc > tok:
                    r = lrow >> 8
                    if self.info[r] & INFO_COUNT:
                        out.append((int(self.kind[r]), lacc - tok, tok))
                    tok, st = lacc, 0
                    p = tok
                    while p < upto:
                        step(w[p], p)
                        p += 1
                        if st == self.fail:
                            break
                else:
                    st = self.sink

        def step(b, p):
            nonlocal st, tok, lacc, lrow
            x = int(T[st + (b ^ ((st >> 8) & 31))])
            if x & EMIT:
                if x & COUNT:
                    out.append(((x >> 24) & 0xFF, p - tok, tok))
                tok = p
            st = (x & ROWMASK) >> 2
            if x & ACC:
                lacc, lrow = p + 1, st

        for p in range(s, e):
            step(w[p], p)
            if not self.mono and st == self.fail:
                recover(p + 1)
        while True:
            if not self.mono and st == self.fail:
                recover(e)
                continue
            if st == 0:
                return out, None
            if st == self.sink:
                return out, tok
            r = st >> 8
            if self.info[r] & INFO_ACC:
                if self.info[r] & INFO_COUNT:
                    out.append((int(self.kind[r]), e - tok, tok))
                return out, None
            if self.mono:
                return out, tok
            st = self.fail

    def scan(self, w: bytes, cuts):
        """Chunked scan with the first-halted-slice truncation; returns (tokens, error_offset)."""
        bounds = [0] + list(cuts) + [len(w)]
        toks = []
        for a, b in zip(bounds, bounds[1:]):
            t, halt = self.walk(w, a, b)
            toks += t
            if halt is not None:
                return toks, halt
        return toks, len(w)
