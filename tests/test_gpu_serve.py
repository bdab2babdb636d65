"""The serving loop: requests arriving open-loop while others are on the GPU are batched
continuously onto several slots whose work overlaps; each request's result must be exactly
the oracle's scan of that request, and the same as the request's result when it is served
alone (bit-exact: the stated tolerance for this integer path)."""
import numpy as np
import pytest

import oracle
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu

SETS = [(T.CLIKE_L, False), (T.CLIKE_D, True), (T.JSON, True)]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def test_results_same_alone_and_in_the_mix():
    from paper_2608_03473_amd import serve

    pool = serve.make_pool(40, 11, median=4096, hi=256 << 10)
    # a few malformed requests: the error offset travels with the result
    for i in (3, 50, 97):
        inst, b = pool[i]
        b = b.copy()
        b[len(b) // 2] = 1
        pool[i] = (inst, b)
    server = serve.Server(serve.instances(), budget_bytes=2 << 30, slots=3, max_docs=512, slot_cap=8 << 20)
    # about 400 requests in 0.4 s: several arrive while every slot is busy
    metrics, done = serve.open_loop(server, pool, 1000.0, 0.4, seed=3, keep=True)
    print(f"[case] serving mix: {metrics}", flush=True)
    assert metrics["requests"] == len(done) > 300 and metrics["errors"] == 0
    assert metrics["batch_size_max"] > 1  # requests were batched
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in SETS]
    want = {}
    for r in done:
        key = id(r.payload)
        if key not in want:
            defs, disc = SETS[r.inst]
            k, l, con = orcs[r.inst].lex(bytes(r.payload), discard=disc)
            want[key] = (k, l, con)
        k, l, con = want[key]
        assert r.status == 0 and r.error_offset == con, (r.rid, r.inst)
        np.testing.assert_array_equal(r.kinds, k, err_msg=f"request {r.rid}")
        np.testing.assert_array_equal(r.lens, l, err_msg=f"request {r.rid}")
    # the same requests one at a time
    alone = serve.Server(serve.instances(), budget_bytes=1 << 30, slots=1, max_docs=1, slot_cap=8 << 20)
    for r in done[:60]:
        alone.admit(serve.Request(r.rid, r.inst, r.payload, 0.0), 0.0)
        out = []
        while alone.busy():
            out += alone.step(lambda: 0.0)
        (a,) = out
        assert (a.ntokens, a.error_offset, a.status) == (r.ntokens, r.error_offset, r.status)
        np.testing.assert_array_equal(a.kinds, r.kinds)
        np.testing.assert_array_equal(a.lens, r.lens)


def test_slots_overlap_under_load():
    """At a high arrival rate more than one slot is busy at once (continuous batching, not a
    queue in front of one launch)."""
    from paper_2608_03473_amd import serve

    pool = serve.make_pool(64, 12, median=8192, hi=1 << 20)
    server = serve.Server(serve.instances(), budget_bytes=2 << 30, slots=3, max_docs=256, slot_cap=4 << 20)
    metrics = serve.open_loop(server, pool, 20000.0, 0.5, seed=4)
    print(f"[case] serving load: {metrics}", flush=True)
    assert metrics["errors"] == 0 and metrics["max_slots_busy"] >= 2
    assert metrics["p50_us"] is not None and metrics["p99_us"] >= metrics["p50_us"]


def test_large_batches_split_by_views():
    """Many requests admitted at once go out as large batches (gathered and split with one
    numpy call each, requests holding views of the batch's tokens): every result is the
    oracle's scan of its request."""
    from paper_2608_03473_amd import serve

    pool = serve.make_pool(30, 13, median=2048, hi=64 << 10)
    server = serve.Server(serve.instances(), budget_bytes=1 << 30, slots=2, max_docs=64, slot_cap=4 << 20)
    for i, (inst, b) in enumerate(pool):
        server.admit(serve.Request(i, inst, b, 0.0), 0.0)
    done = []
    while server.busy():
        done += server.step(lambda: 0.0)
    print(f"[case] serving large batches: sizes {server.batch_sizes}", flush=True)
    assert len(done) == len(pool) and max(server.batch_sizes) > serve._SMALL
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in SETS]
    for r in done:
        defs, disc = SETS[r.inst]
        k, l, con = orcs[r.inst].lex(bytes(r.payload), discard=disc)
        assert r.status == 0 and r.error_offset == con and r.ntokens == len(k), r.rid
        np.testing.assert_array_equal(r.kinds, k, err_msg=f"request {r.rid}")
        np.testing.assert_array_equal(r.lens, l, err_msg=f"request {r.rid}")


def test_admission_against_the_budget():
    """Every slot's device memory (input, worst-case outputs, document records, workspace)
    fits the HBM budget; a request larger than a slot is refused with LEX_ELIMIT and one
    arriving while the waiting queue is full with LEX_ENOMEM, each at once and with no
    tokens, while every admitted request still equals the oracle's scan."""
    from paper_2608_03473_amd import serve

    budget = 64 << 20
    server = serve.Server(serve.instances(), budget_bytes=budget, slots=2, max_docs=64, slot_cap=1 << 20,
                          max_pending_bytes=256 << 10)
    assert server.reserved_bytes <= budget and server.slot_bytes <= 1 << 20
    pool = serve.make_pool(20, 14, median=16384, hi=128 << 10)
    big = (0, np.frombuffer(b"x = 1;\n" * ((server.slot_bytes // 7) + 10), np.uint8).copy())
    reqs = [serve.Request(i, inst, b, 0.0) for i, (inst, b) in enumerate(pool)]
    reqs.append(serve.Request(len(reqs), big[0], big[1], 0.0))
    admitted = [server.admit(r, 0.0) for r in reqs]
    assert not admitted[-1] and reqs[-1].status == P.LEX_ELIMIT
    assert not all(admitted[:-1])  # the queue bound refused some of the pool
    done = []
    while server.busy():
        done += server.step(lambda: 0.0)
    print(f"[case] serving admission: slot {server.slot_bytes} B, reserved {server.reserved_bytes} B, "
          f"refused {sum(not a for a in admitted)}", flush=True)
    assert len(done) == len(reqs)
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in SETS]
    for r, ok in zip(reqs, admitted):
        if not ok:
            assert r.status in (P.LEX_ELIMIT, P.LEX_ENOMEM) and r.ntokens == 0 and r.kinds.size == 0
            continue
        defs, disc = SETS[r.inst]
        k, l, con = orcs[r.inst].lex(bytes(r.payload), discard=disc)
        assert r.status == 0 and r.error_offset == con and r.ntokens == len(k), r.rid
        np.testing.assert_array_equal(r.kinds, k, err_msg=f"request {r.rid}")
        np.testing.assert_array_equal(r.lens, l, err_msg=f"request {r.rid}")
