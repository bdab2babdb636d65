"""The whole-stream manifest (tests/golden/stream_manifest.json) against its sources, on
the CPU: every benchmark corpus regenerates to the digest recorded with the oracle's
output (a drifted generator would otherwise surface as a GPU mismatch), the stray-byte
draws are the ones the recorded rule picks, and the oracle reproduces the recorded
digests of the 1 MiB configuration.  The GPU tests compare the device's whole output with
the same digests."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import stream_manifest as SM  # noqa: E402

MAN = SM.load()["cases"]


def test_manifest_covers_the_benchmark_configurations():
    assert set(MAN) == set(SM.CASES)
    for name, case in MAN.items():
        for k, v in SM.CASES[name].items():
            assert case[k] == v, (name, k)
    assert MAN["clike_512mib"]["error_offset"] == 512 << 20
    assert MAN["json_256mib"]["error_offset"] == 256 << 20
    assert MAN["clike_512mib_stray_error"]["error_offset"] < 512 << 20
    assert MAN["clike_512mib_stray_ok"]["ntokens"] == MAN["clike_512mib"]["ntokens"]
    assert MAN["docs_50k"]["incomplete_documents"] == 0
    for name in ("clikeb_512mib_framed", "clikeb_512mib"):
        assert MAN[name]["error_offset"] == 512 << 20
    # the framed corpus differs from the unframed one by its separators, each a token
    assert MAN["clikeb_512mib_framed"]["ntokens"] > MAN["clikeb_512mib"]["ntokens"]


@pytest.mark.parametrize("name", ["clike_1mib", "json_256mib", "clikeb_512mib_framed", "clikeb_512mib"])
def test_corpus_digest(name):
    assert SM.sha(SM.corpus(MAN[name])) == MAN[name]["corpus_sha256"]


def test_clike_512mib_corpus_and_stray_draws():
    case = MAN["clike_512mib"]
    buf = SM.corpus(case)
    assert SM.sha(buf) == case["corpus_sha256"]
    oc = oracle.OracleSet(T.as_tuples(T.CLIKE_L))
    for name in ("clike_512mib_stray_error", "clike_512mib_stray_ok"):
        s = MAN[name]
        draw, x = SM.pick_stray(buf, oc, s["stray_seed"], s["want_error"])
        assert (draw, x) == (s["stray_draw"], s["stray_offset"]), name
        old = buf[x]
        buf[x] = 1
        assert SM.sha(buf) == s["stray_corpus_sha256"], name
        buf[x] = old


@pytest.mark.slow
def test_docs_corpus_digest():
    case = MAN["docs_50k"]
    sizes, sets = workloads.doc_plan(case["count"], case["seed"])
    assert SM.sha(sizes.astype("<u8")) == case["sizes_sha256"]
    assert SM.sha(sets) == case["sets_sha256"]
    buf, _, _, _ = SM.corpus(case)
    assert buf.size == case["nbytes"] and SM.sha(buf) == case["corpus_sha256"]


def test_oracle_reproduces_the_1mib_digests():
    case = MAN["clike_1mib"]
    k, l, con = oracle.OracleSet(T.as_tuples(T.CLIKE_L)).lex(SM.corpus(case))
    assert (k.size, con) == (case["ntokens"], case["error_offset"])
    d = SM.stream_digest(k, l)
    assert (d["kinds"], d["lens"], d["blocks"]) == (case["kinds"], case["lens"], case["blocks"])


def test_digest_localises_a_difference():
    """A planted difference in one token is caught by the whole digest and localised to its
    block."""
    rng = np.random.default_rng(3)
    k = rng.integers(0, 7, 3 * SM.BLOCK_TOKENS + 11).astype(np.uint8)
    l = rng.integers(1, 40, k.size).astype(np.uint32)
    want = SM.stream_digest(k, l)
    l2 = l.copy()
    l2[2 * SM.BLOCK_TOKENS + 5] += 1
    got = SM.stream_digest(k, l2)
    assert got["kinds"] == want["kinds"] and got["lens"] != want["lens"]
    assert SM.first_bad_block(want["blocks"], got["blocks"]) == 2
    assert SM.first_bad_block(want["blocks"], want["blocks"]) == -1
    assert SM.first_bad_block(want["blocks"], want["blocks"][:2]) == 2
