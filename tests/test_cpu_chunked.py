"""The host baseline (lex_cpu_chunked: the paper's multithreaded chunked executor of
Section 6 on the CPU cores) against the oracle's serial scan, element by element.

By Theorem 1 (exact mode) and Theorem 3 (modulo I) the chunked scan over certified cuts
equals the serial scan; on malformed input the output stops after the first halting chunk
with con(w) as error offset (Corollary 1).  Cases: every benchmark token set in its
mode, chunk lengths from 64 bytes (many chunks, cuts sliding past targets) to the 64 KiB
default, 1, 3 and 8 threads, ragged sizes, stray bytes, the serial mode, a refused set
(one chunk), empty input, and random token sets over small alphabets."""
import random

import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T
from randsets import rand_set

P = pytest.importorskip("paper_2608_03473_amd")

EXACT, DISCARD, SERIAL = 0, 1, 2


def _check(defs, buf, mode, chunk, threads):
    lx = P.Lexer.compile(defs)
    k, l, nt, err, nch = lx.cpu_chunked(buf, mode, chunk_bytes=chunk, threads=threads)
    ok, ol, con = oracle.OracleSet(defs).lex(bytes(buf), discard=bool(mode & 1))
    assert err == con and nt == ok.size
    np.testing.assert_array_equal(k, ok)
    np.testing.assert_array_equal(l, ol)
    return nch


GENS = {
    "clike_l": (lambda n, s: workloads.clike(n, s), EXACT),
    "clike_d": (lambda n, s: workloads.clike(n, s), DISCARD),
    "clike_b": (lambda n, s: workloads.clike(n, s, bcomment=True), DISCARD),
    "json": (lambda n, s: workloads.json(n, s), DISCARD),
    "log": (lambda n, s: workloads.loglines(n, 40), EXACT),
}


@pytest.mark.parametrize("name", sorted(GENS))
@pytest.mark.parametrize("chunk,threads", [(64, 3), (4096, 8), (64 << 10, 1)])
def test_benchmark_sets(name, chunk, threads):
    gen, mode = GENS[name]
    defs = T.as_tuples(T.NAMED[name])
    nch = _check(defs, gen((1 << 20) + 37, 9), mode, chunk, threads)
    cert = P.Lexer.compile(defs).cert(mode)
    if cert:
        assert nch > 1
    else:
        assert nch == 1  # a refused set runs as one chunk


@pytest.mark.parametrize("mode", [EXACT, SERIAL])
def test_stray_bytes_truncate_at_the_first_halting_chunk(mode):
    """Corollary 1: stray 0x01 bytes outside strings and comments halt the scan at the
    first of them; every token before it is kept."""
    defs = T.as_tuples(T.CLIKE_L)
    buf = workloads.clike(300000, 4)
    rng = np.random.default_rng(1)
    for x in sorted(rng.integers(1000, buf.size, 6)):
        buf[x] = 1
    _check(defs, buf, mode, 256, 4)


def test_json_exact_mode_and_tails():
    """JSON (non-monotone: the number '1.' backs off) in exact mode (no certified byte, one
    chunk) and a JSON buffer cut in the middle of a value (the tail halts)."""
    defs = T.as_tuples(T.JSON)
    buf = workloads.json(200000, 2)
    _check(defs, buf, EXACT, 512, 3)
    _check(defs, buf[:123457], DISCARD, 512, 3)


def test_empty_and_tiny_inputs():
    defs = T.as_tuples(T.CLIKE_L)
    for data in (b"", b"\n", b"a", b"&", b"x \n\n\n"):
        _check(defs, np.frombuffer(data, np.uint8), EXACT, 16, 2)


@pytest.mark.parametrize("seed", range(40))
def test_random_sets(seed):
    """Random token sets over {a, b, c, ;}: the chunked scan at 16-byte chunks equals the
    serial scan in both modes, on valid and malformed strings."""
    defs = rand_set(1000 + seed, "abc;")
    try:
        lx = P.Lexer.compile(defs)
    except P.LexError:
        pytest.skip("set does not compile (empty language)")
    rng = random.Random(seed)
    for trial in range(4):
        s = "".join(rng.choice("abc;") for _ in range(rng.randint(0, 600)))
        buf = np.frombuffer(s.encode(), np.uint8)
        for mode in (EXACT, DISCARD):
            k, l, nt, err, _ = lx.cpu_chunked(buf, mode, chunk_bytes=16, threads=3)
            ok, ol, con = oracle.OracleSet(defs).lex(s.encode(), discard=bool(mode))
            assert (nt, err) == (ok.size, con), (defs, s, mode)
            np.testing.assert_array_equal(k, ok)
            np.testing.assert_array_equal(l, ol)


def test_argument_checks():
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    buf = workloads.clike(1000, 1)
    with pytest.raises(P.LexError):
        lx.cpu_chunked(buf, 0, kinds=np.empty(999, np.uint8), lens=np.empty(999, np.uint32))
    with pytest.raises(P.LexError):
        lx.cpu_chunked(buf, 7)
