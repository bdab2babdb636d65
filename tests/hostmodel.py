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
        # some token end of this mode is not counted (a discarded kind)
        self.disc = bool((((self.T & EMIT) != 0) & ((self.T & COUNT) == 0)).any())
        self.fail = self.sink if self.mono else (2 + inf["nstates"]) * 256

    def walk(self, w: bytes, s: int, e: int, memo: int = 4, work=None):
        """Tokens (kind, length, start) written by a lane on [s, e), and its halt offset or None.
        memo: failed traces kept by the fallback (0: plain re-scans); work: a one-element list
        that receives the transitions taken (walk, re-scans and failed-trace cursors)."""
        T, out = self.T, []
        st, tok, lacc, lrow = 0, s, s, 0
        steps = 0

        def nxt(row, b):
            return (int(T[row + (b ^ ((row >> 8) & 31))]) & ROWMASK) >> 2

        def recover(upto):  # non-monotone automata only (FAIL != SINK)
            nonlocal st, tok, lacc, lrow, steps
            # failed traces as cursors [position, row]: every (row, position) pair a trace visits
            # after its last accepting step leads to FAIL, or to the end of the slice, without
            # another accepting state
            segs = []
            while st == self.fail:
                if lacc > tok:
                    if memo:
                        if len(segs) == memo:
                            segs.pop(0)
                        segs.append([lacc, lrow])
                    r = lrow >> 8
                    if self.info[r] & INFO_COUNT:
                        out.append((int(self.kind[r]), lacc - tok, tok))
                    tok, st = lacc, 0
                    p = tok
                    while p < upto:
                        step(w[p], p)
                        for c in segs:
                            if c[0] == p:
                                c[0], c[1] = p + 1, nxt(c[1], w[p])
                                steps += 1
                        segs = [c for i, c in enumerate(segs) if c[1] != self.fail and c not in segs[:i]]
                        p += 1
                        if st == self.fail:
                            break
                        if any(c[0] == p and c[1] == st for c in segs):
                            st = self.fail  # a failed pair: this trace fails as that one did
                            break
                else:
                    st = self.sink

        def step(b, p):
            nonlocal st, tok, lacc, lrow, steps
            steps += 1
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
            if work is not None:
                work[0] = steps
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


def plan_cuts(w: bytes, cert, lane: int):
    """Lane boundaries c(j l) (c(0) = 0, c(x) = first certified byte at or after x, or n)."""
    n = len(w)
    nl = max(1, -(-n // lane))
    nxt = [n] * (n + 1)
    for i in range(n - 1, -1, -1):
        nxt[i] = i if w[i] in cert else nxt[i + 1]
    cuts = [0] + [nxt[min(j * lane, n)] for j in range(1, nl)] + [n]
    return cuts


def plan_fused(w: bytes, cert, lane: int):
    """Slice starts and ends as the fused planner records them: lane j searches [j l, (j+1) l)
    for a certified byte; without one its slice is empty at min(j l, n); a slice ends at the
    next lane's start or, when that lane found none, at the first certified byte after it."""
    n = len(w)
    nl = max(1, -(-n // lane))
    first = []
    for j in range(nl):
        if j == 0:
            first.append(0)
            continue
        hit = next((p for p in range(j * lane, min((j + 1) * lane, n)) if w[p] in cert), None)
        first.append(hit)
    starts, ends = [], []
    for j in range(nl):
        if first[j] is None:
            starts.append(min(j * lane, n))
            ends.append(min(j * lane, n))
            continue
        starts.append(first[j])
        if j + 1 == nl or (j + 1) * lane >= n:
            ends.append(n)
        elif first[j + 1] is not None:
            ends.append(first[j + 1])
        else:
            ends.append(next((p for p in range((j + 1) * lane, n) if w[p] in cert), n))
    return starts, ends


def windowed(model, w: bytes, starts, ends, lane: int, base: int, block: int = 4,
             stage_words: int = 1280, W: int = 64, offsets: bool = True):
    """The checkpointed count walk and the windowed emit of the library, restated.

    starts/ends: the lanes' slices (lane j nominally covers [j l, (j+1) l)).  base: the
    input's address modulo W.  block: lanes per count workgroup.  Returns (kinds, lens, offs),
    or None when a slice halts (the library then uses the lane emit).  Mirrors the kernels'
    bookkeeping: window checkpoints, owner lookup through the last-non-empty-lane prefixes,
    64-window tiles, the staged words (end - P) << 8 | kind after 4 to 7 padding slots (in a
    mode with discarded kinds, length << 8 | kind, and no staging when offsets are asked
    for), and the direct fallback for ranges longer than the stage.  Without offsets the
    third list is None.
    """
    disc = model.disc
    T, info, kind = model.T, model.info, model.kind
    n, nl, mis0 = len(w), len(starts), base % W
    kslots = lane // W + 4
    counts, nonempty, ck = [0] * nl, [False] * nl, {}

    def ent(st, b):
        return int(T[st + (b ^ ((st >> 8) & 31))])

    for j in range(nl):
        s, e = starts[j], ends[j]
        nonempty[j] = s < e
        st, cnt, tok = 0, 0, s
        for p in range(s, e):
            if p > s and (base + p) % W == 0:
                # main slots by (window within the lane's nominal range, lane), else overflow
                k = (p - j * lane) // W
                ck[(k, j) if k < kslots else ("over", (p + mis0) // W)] = (st >> 8, cnt, tok)
            x = ent(st, w[p])
            cnt += x & COUNT
            if x & EMIT:
                tok = p
            st = (x & ROWMASK) >> 2
        if st != 0:
            r = st >> 8
            if st == model.sink or not (info[r] & INFO_ACC):
                return None  # halted slice
            if info[r] & INFO_COUNT:
                cnt += 1
        counts[j] = cnt
    nb = -(-nl // block)
    lane_pre, lnz, blk_sum, blk_lnz = [0] * nl, [-1] * nl, [0] * nb, [-1] * nb
    run, zrun = 0, -1
    for b in range(nb):
        blk_sum[b], blk_lnz[b] = run, zrun
        acc, z = 0, -1
        for j in range(b * block, min(nl, (b + 1) * block)):
            lane_pre[j] = acc
            acc += counts[j]
            if nonempty[j]:
                z = j
            lnz[j] = z
        run += acc
        zrun = max(zrun, z)
    ntok = run
    nwin = -(-(n + mis0) // W) if n else 0

    def meta(i):
        """(row state, token start, output offset, a lane starts here) at window i's start."""
        if i >= nwin:
            return 0, 0, ntok, False
        ws = i * W - mis0 if i else 0
        j0 = min(ws // lane, nl - 1)
        here = starts[j0] < ends[j0] and starts[j0] <= ws
        owner = j0 if here else (lnz[j0 - 1] if lnz[j0 - 1] >= 0 else blk_lnz[(j0 - 1) // block])
        off = blk_sum[owner // block] + lane_pre[owner]
        if here and starts[j0] == ws:
            return 0, ws, off, True
        k = (ws - owner * lane) // W
        r, run, tok = ck[(k, owner) if k < kslots else ("over", i)]
        return r * 256, tok, off + run, False

    kinds, lens, offs = [None] * ntok, [None] * ntok, [None] * ntok
    for tile in range(-(-nwin // 64)):
        ids = [tile * 64 + L for L in range(64)]
        ms = [meta(i) for i in ids]
        nxt = [meta(i + 1) for i in ids]
        o_first = ms[0][2]
        last = min(63, nwin - 1 - tile * 64)
        o_end = nxt[last][2]
        P = ms[0][1]
        total, pad = o_end - o_first, (o_first & 3) + 4
        span_end = min((tile + 1) * 64 * W - mis0, n)
        staged = (o_first <= o_end <= ntok and total + pad + 3 <= stage_words - 64 and span_end - P < (1 << 24)
                  and not (disc and offsets))
        stage = {pad - 1: 0}  # the end before the tile's first token: 0 relative to P
        for L, i in enumerate(ids):
            if i >= nwin:
                continue
            st, tok, out, _ = ms[L]
            lim = min(nxt[L][2], ntok)
            slot, o = pad + out - o_first, out
            for p in range(max(0, i * W - mis0), min(n, i * W - mis0 + W)):
                y = ent(st, w[p])
                if staged:
                    if y & COUNT:
                        v = p - tok if disc else p - P
                        stage[slot] = ((v & 0xFFFFFF) << 8) | ((y >> 24) & 0xFF)
                        slot += 1
                else:
                    if (y & COUNT) and o < lim:
                        kinds[o], lens[o], offs[o] = (y >> 24) & 0xFF, p - tok, tok
                        o += 1
                if y & EMIT:
                    tok = p
                st = (y & ROWMASK) >> 2
            # the input's end, or a lane starting at the next window: the token ends here
            if (i + 1 == nwin or nxt[L][3]) and st != 0:
                end = n if i + 1 == nwin else (i + 1) * W - mis0
                r = st >> 8
                if (info[r] & INFO_ACC) and (info[r] & INFO_COUNT):
                    if staged:
                        stage[slot] = int(kind[r]) | ((end - (tok if disc else P)) << 8)
                    elif o < lim:
                        kinds[o], lens[o], offs[o] = int(kind[r]), end - tok, tok
        if not staged:
            continue
        o0 = o_first - pad
        for q in range(4, pad + total, 4):
            ev = [stage.get(g, 0) >> 8 for g in range(q - 1, q + 4)]
            for k in range(4):
                g = q + k
                if pad <= g < pad + total:
                    if disc:  # the word holds the length; no offsets in this form
                        kinds[o0 + g], lens[o0 + g], offs[o0 + g] = stage[g] & 0xFF, ev[k + 1], None
                    else:
                        kinds[o0 + g], lens[o0 + g], offs[o0 + g] = stage[g] & 0xFF, ev[k + 1] - ev[k], P + ev[k]
    return kinds, lens, (offs if offsets else None)


def spec_walk(model, w: bytes, b: int, end: int):
    """The hybrid plan's speculative walk of [b, end): from the start row as if a token began
    at b, restarting one byte further on after a halt.  Returns (token starts, last restart
    or None)."""
    T = model.T
    st, tok, lacc, p, rst = 0, b, b, b, None
    starts = [b]
    while p < end:
        x = int(T[st + (w[p] ^ ((st >> 8) & 31))])
        if x & EMIT:
            tok = p
            starts.append(p)
        st = (x & ROWMASK) >> 2
        if not model.mono and (x & ACC):
            lacc = p + 1
        p += 1
        if st == model.sink or (not model.mono and st == model.fail):
            if not model.mono and st == model.fail and lacc > tok:
                tok = lacc
            else:
                rst, tok = tok, tok + 1
            p, lacc, st = tok, tok, 0
            if p < end:
                starts.append(p)
    return starts, rst


def spec_plan(model, w: bytes, S: int, X: int):
    """Cuts of the hybrid plan for a document of a refused set: lane k walks [k S, (k+1) S + X)
    speculatively; cut k is the first position in [k S, k S + X) that starts a token in both
    lane k-1's walk and lane k's (for the last lane, whose window reaches the end, the end when
    there is none: lane k-1's walk is then the serial scan up to the end).  None when a cut is
    missing or a lane restarted at or after its own cut (the document then runs on one lane)."""
    n = len(w)
    m = -(-n // S)
    walks = [spec_walk(model, w, k * S, min((k + 1) * S + X, n)) for k in range(m)]
    cuts = [0]
    for k in range(1, m):
        common = sorted(set(t for t in walks[k - 1][0] if k * S <= t < k * S + X) &
                        set(t for t in walks[k][0] if t < k * S + X))
        if not common and k == m - 1:
            common = [n]  # lane k - 1's walk reached the end: it takes the rest
        if not common:
            return None
        cuts.append(common[0])
    for k in range(m):
        rst = walks[k][1]
        if rst is not None and rst >= cuts[k]:
            return None
    return cuts


def spec_parts(model, w: bytes, S: int, cuts, parts: int = 4):
    """The batch's split of each hybrid-plan slice [s, e) into `parts` walks (S = the sync
    window = the speculative lane): part q > 0 starts at the first token start of lane k's
    speculative walk at or after s + q (e - s) // parts and before e, looked up only where
    the walk marked them (head [k S, (k+1) S), tail [(k+1) S, (k+2) S)), else at e.  Returns
    per slice the list of part starts (parts entries, the first being s)."""
    n = len(w)
    out = []
    for k, (s, e) in enumerate(zip(cuts, cuts[1:] + [n])):
        starts, _ = spec_walk(model, w, k * S, min((k + 1) * S + S, n))
        b2 = min((k + 1) * S, n)
        marked = sorted(t for t in starts if (k * S <= t < k * S + S) or (b2 <= t < b2 + S))
        ps = [s]
        for q in range(1, parts):
            x = s + (e - s) * q // parts
            ps.append(next((t for t in marked if x <= t < e), e))
        out.append(ps)
    return out
