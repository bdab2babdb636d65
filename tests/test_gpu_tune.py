"""Every configuration the autotuner may choose writes the oracle's stream: each candidate
(one pass, fused and pipeline paths at several lane targets and block sizes, the lane emit)
on a C-like corpus in exact mode and a JSON corpus modulo I, and every batch-lane candidate
on a mixed batch, compared element by element with the oracle's serial scan (Theorems 1 and
3).  Then one tuning run, whose choice is one of those candidates."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
from paper_2608_03473_amd import tune  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


CASES = [("clike_l", lambda: workloads.clike((3 << 20) + 41, 21), P.LEX_MODE_EXACT),
         ("json", lambda: workloads.json((2 << 20) + 7, 22), P.LEX_MODE_DISCARD)]


@pytest.mark.parametrize("name,gen,mode", CASES, ids=[c[0] for c in CASES])
def test_every_candidate_equals_the_oracle(name, gen, mode, tmp_path):
    defs = T.as_tuples(T.NAMED[name])
    lx, oc = P.Lexer.compile(defs), oracle.OracleSet(defs)
    buf = gen()
    k, l, con = oc.lex(buf, discard=bool(mode))
    data = torch.from_numpy(buf).cuda()
    tu = tune.Tuner(cache_path=str(tmp_path / "t.json"), reps=2)
    cands = tu.candidates(lx, buf.size, mode, 64 << 10)
    print(f"[case] tune {name}: {len(cands)} candidates", flush=True)
    for o, plan in cands:
        r = lx.run(data, mode=mode, opts=o)
        assert (r.status, r.error_offset, r.ntokens) == (0, con, k.size), plan
        np.testing.assert_array_equal(r.kinds.cpu().numpy(), k, err_msg=str(plan))
        np.testing.assert_array_equal(r.lens.cpu().numpy().view(np.uint32), l, err_msg=str(plan))
    e = tu.tune(lx, data, mode, 64 << 10)
    assert e["opts"] in [tune.opts_dict(o) for o, _ in cands] and e["ms"] <= e["default_ms"]
    assert tu.best(lx, buf.size, mode, 64 << 10) is not None


def test_batch_lane_candidates_equal_the_oracle(tmp_path):
    insts = [(T.CLIKE_L, P.LEX_MODE_EXACT), (T.CLIKE_D, P.LEX_MODE_DISCARD), (T.CLIKE_B, P.LEX_MODE_DISCARD)]
    buf, offs, sizes, sets = workloads.docs(300, 23)
    lms = [(P.Lexer.compile(T.as_tuples(d)), m) for d, m in insts]
    batch = P.Batch(lms)
    docs = np.zeros(sizes.size, dtype=P.DOC_DTYPE)
    docs["offset"], docs["length"], docs["inst"] = offs, sizes, sets
    orcs = [oracle.OracleSet(T.as_tuples(d)) for d, _ in insts]
    want = [orcs[s].lex(bytes(buf[int(o):int(o) + int(z)]), discard=bool(insts[s][1]))
            for o, z, s in zip(offs, sizes, sets)]
    data = torch.from_numpy(buf).cuda()
    for lane in tune.BATCH_LANES:
        print(f"[case] batch lane {lane}", flush=True)
        r = batch.run(data, docs, opts=P.RunOpts(lane_bytes=lane))
        assert r.status == 0
        for i, (k, l, con) in enumerate(want):
            t0, nt = int(r.docs["tok_offset"][i]), int(r.docs["ntokens"][i])
            assert nt == k.size and int(r.docs["error_offset"][i]) == con, (lane, i)
            np.testing.assert_array_equal(r.kinds[t0:t0 + nt].cpu().numpy(), k, err_msg=f"lane {lane} doc {i}")
            np.testing.assert_array_equal(r.lens[t0:t0 + nt].cpu().numpy().view(np.uint32), l)
    tu = tune.Tuner(cache_path=str(tmp_path / "t.json"), reps=2)
    docs_dev = torch.from_numpy(docs.view(np.uint8).copy()).cuda()
    e = tu.tune_batch(batch, lms, data, docs_dev, sizes.size)
    assert e["ms"] <= e["default_ms"]
