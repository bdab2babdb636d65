"""Bounded failed lookahead on the GPU: inputs on which naive longest match re-scans the same
bytes over and over (Section 9's a^N over {a, a+b, ;}, where ';' certifies but never occurs
so the plan is one slice; unterminated block comments of the C-like-B set).  Parity with the
oracle where the oracle (itself a plain re-scanning lexer) finishes quickly, and with the
closed form it pins at larger sizes; scan times are printed and bounded far below what
quadratic re-scans would take.
"""
import time

import numpy as np
import pytest

import oracle
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu

EX = [("a", 0, False), ("a+b", 0, False), (";", 0, False)]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def run_timed(lx, w, mode=0, opts=None):
    dev = torch.from_numpy(np.frombuffer(w, np.uint8).copy()).cuda()
    lx.run(dev, mode=mode, opts=opts)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = lx.run(dev, mode=mode, offsets=True, opts=opts)
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def test_paper_example_one_slice():
    lx = P.Lexer.compile(EX)
    assert lx.cert() == {ord(";")}
    oc = oracle.OracleSet(EX)
    k, l, con = oc.lex(b"a" * 2048)
    assert con == 2048 and (k == 0).all() and (l == 1).all()  # the closed form, pinned
    for n in (2048, 16384):
        print(f"[case] a^{n} over {{a, a+b, ;}}", flush=True)
        r, dt = run_timed(lx, b"a" * n)
        print(f"  {n} bytes: {dt * 1e3:.2f} ms, {r.nslices} slice(s)", flush=True)
        assert r.status == 0 and r.error_offset == n and r.ntokens == n and r.nslices == 1
        assert (r.kinds.cpu().numpy() == 0).all() and (r.lens.cpu().numpy() == 1).all()
        np.testing.assert_array_equal(r.offsets.cpu().numpy(), np.arange(n))
        assert dt < 2.0


UNITS = [b"/*a", b"/*a\n", b"/*\t", b"/**a"]


@pytest.mark.parametrize("unit", UNITS)
def test_unterminated_block_comments(unit):
    """Every '/*' opens a comment that never closes: each one makes naive longest match scan
    to the end of the slice and fall back.  Refused set: one lane, the serial mode, and the
    hybrid plan (speculative walks) once the input passes one speculative lane."""
    defs = T.as_tuples(T.CLIKE_B)
    lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
    small = unit * 600
    for mode in (P.LEX_MODE_EXACT, P.LEX_MODE_DISCARD):
        k, l, o, con = oc.lex(small, discard=bool(mode), offsets=True)
        period = len(k) // 600
        assert len(k) == 600 * period and con == len(small)
        # the stream is one period per unit (checked here by the oracle), so the closed form
        # below holds at any number of units
        np.testing.assert_array_equal(k, np.tile(k[:period], 600))
        np.testing.assert_array_equal(l, np.tile(l[:period], 600))
        for m in (mode, mode | P.LEX_MODE_SERIAL):
            print(f"[case] {unit!r} x600 mode={m}", flush=True)
            r, _ = run_timed(lx, small, m)
            assert r.status == 0 and r.error_offset == con and r.ntokens == len(k)
            np.testing.assert_array_equal(r.kinds.cpu().numpy(), k)
            np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l)
            np.testing.assert_array_equal(r.offsets.cpu().numpy().astype(np.uint64), o)
        reps = 6000
        big = unit * reps
        for m in (mode, mode | P.LEX_MODE_SERIAL):
            print(f"[case] {unit!r} x{reps} mode={m}", flush=True)
            r, dt = run_timed(lx, big, m)
            print(f"  {len(big)} bytes: {dt * 1e3:.2f} ms, {r.nslices} slice(s)", flush=True)
            assert r.status == 0 and r.error_offset == len(big) and r.ntokens == reps * period
            np.testing.assert_array_equal(r.kinds.cpu().numpy(), np.tile(k[:period], reps))
            np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), np.tile(l[:period], reps))
            assert dt < 2.0
