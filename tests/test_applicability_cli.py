"""The applicability CLI (CPU only): run on the Table 2 transcriptions it must reproduce the
table's useful certified sets (the golden fixture, which cites Table 2), through the
library's own compiler; on a token-set file it must report both modes and what the scan
does with them."""
import json
import os

import pytest

from paper_2608_03473_amd import applicability
from workloads import tokensets as T

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_applicability.json")


def test_table2_through_the_cli(capsys):
    assert applicability.main(["--json"]) == 0
    got = {}
    for line in capsys.readouterr().out.splitlines():
        r = json.loads(line)
        got[r["set"]] = r
    g = json.load(open(GOLDEN))
    ops = {ord(c) for c in T.ROW1_OPS}
    expand = lambda v: ops if v == "ops24" else ops | {9, 10, 32} if v == "ops24+[9,10,32]" else set(v)  # noqa: E731
    assert {row["set"] for row in g["rows"]} <= set(got)
    for row in g["rows"]:
        r = got[row["set"]]
        assert set(r["exact"]["useful"]) == expand(row["exact"]), row["row"]
        assert set(r["discard"]["useful"]) == expand(row["modulo"]), row["row"]
        # a useful certified byte is certified (Definition 2 / 3 restricted to useful ones)
        assert set(r["exact"]["useful"]) <= set(r["exact"]["certified"])
        assert set(r["discard"]["useful"]) <= set(r["discard"]["certified"])
    assert "hybrid plan" in got["TABLE2_ROW4_BCOMMENT"]["discard"]["scan"]
    assert got["LOG"]["exact"]["scan"].startswith("splits")


def test_token_set_file(tmp_path, capsys):
    f = tmp_path / "set.json"
    f.write_text(json.dumps([{"name": "WORD", "pattern": "[a-z]+"}, {"name": "SP", "pattern": " ", "discard": True},
                             {"name": "NL", "pattern": "\n"}]))
    assert applicability.main([str(f)]) == 0
    out = capsys.readouterr().out
    assert "set.json" in out and "exact (E, E_u)" in out and "modulo I (D, D_u)" in out
    assert applicability.main(["--json", str(f)]) == 0
    r = json.loads(capsys.readouterr().out)
    assert r["exact"]["useful"] == [10, 32] and r["discard"]["useful"] == [10, 32]
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"pattern": "a"}))
    with pytest.raises(ValueError):
        applicability.main([str(bad)])


def test_reserved_byte_framing(capsys):
    """--reserve 0x1E (Section 7.1): the block-comment row, refused in both modes, certifies
    the reserved byte in both once framed, and its scans split at it."""
    assert applicability.main(["--json", "--reserve", "0x1E"]) == 0
    got = {}
    for line in capsys.readouterr().out.splitlines():
        r = json.loads(line)
        got[r["set"]] = r
    row = got["TABLE2_ROW4_BCOMMENT framed by \\x1E"]
    for mode in ("exact", "discard"):
        assert row[mode]["useful"] == [0x1E] and row[mode]["certified"] == [0x1E]
        assert row[mode]["scan"].startswith("splits")
    # a set that already certified bytes keeps them and adds the reserved one
    assert 0x1E in got["TABLE2_ROW1 framed by \\x1E"]["exact"]["useful"]
    assert len(got["TABLE2_ROW1 framed by \\x1E"]["exact"]["useful"]) > 1
