"""The autotuner's host logic (no scan runs): candidate configurations resolve through
lex_plan, distinct plans are kept once with the defaults first, lanes divide the chunk
length, and options round-trip through the cache's form."""
import pytest

from workloads import tokensets as T

P = pytest.importorskip("paper_2608_03473_amd")
from paper_2608_03473_amd import tune  # noqa: E402


def test_candidates_resolve_and_are_distinct(tmp_path):
    tu = tune.Tuner(cache_path=str(tmp_path / "t.json"))
    for name, mode in (("clike_l", P.LEX_MODE_EXACT), ("json", P.LEX_MODE_DISCARD), ("clike_b", P.LEX_MODE_EXACT)):
        lx = P.Lexer.compile(T.as_tuples(T.NAMED[name]))
        c = tu.candidates(lx, 512 << 20, mode, 64 << 10)
        assert len(c) >= 4
        o0, p0 = c[0]
        assert tune.opts_dict(o0)["lane_bytes"] == 0 and p0 == lx.plan(512 << 20, mode, o0)  # defaults first
        sigs = [(p["lane_bytes"], p["block_threads"], p["path"], p["windowed"], p["hybrid"], o.emit) for o, p in c]
        assert len(sigs) == len(set(sigs))
        for o, p in c:
            assert p == lx.plan(512 << 20, mode, o)
            if o.lane_bytes and not p["hybrid"]:
                assert (64 << 10) % o.lane_bytes == 0
        paths = {p["path"] for _, p in c}
        if name == "clike_l":
            assert paths == {1, 2, 3}  # a monotone set: one pass, fused and the pipeline
        if name == "json":
            assert 3 not in paths  # not monotone: no one pass


def test_options_round_trip():
    o = P.RunOpts(chunk_bytes=65536, lane_bytes=1024, path=2, block_threads=512, emit=1)
    d = tune.opts_dict(o)
    o2 = tune.opts_of(d)
    assert tune.opts_dict(o2) == d
    assert tune.opts_dict(None) == {}
