"""GPU parity of batched document scans (lex_run_batch) against the oracle, document by
document: each document's tokens (kinds, lengths, offsets relative to the document), token
count, error offset and slice count must be those of the oracle's serial scan of that
document alone, whatever its neighbours are (Theorem 1, Theorem 3 per document; Corollary 1
for its truncation).  Also: overflow, a document table the kernels reject, and replays of a
captured CUDA graph against the eager result."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu

INSTANCES = [("clike_l", 0), ("clike_d", 1), ("clike_b", 1), ("json", 1), ("log", 0)]


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def setup():
    lexers = {name: P.Lexer.compile(T.as_tuples(T.NAMED[name])) for name, _ in INSTANCES}
    orcs = {name: oracle.OracleSet(T.as_tuples(T.NAMED[name])) for name, _ in INSTANCES}
    batch = P.Batch([(lexers[n], m) for n, m in INSTANCES])
    return lexers, orcs, batch


def make_docs(count, seed, median=2048):
    """Documents of every instance, log-normal sizes, some empty, some malformed, some serial."""
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.exp(np.log(median) + 1.5 * rng.standard_normal(count)), 0, 96 << 10).astype(np.int64)
    sizes[rng.random(count) < 0.03] = 0
    sizes[rng.random(count) < 0.05] = rng.integers(1, 20)
    parts, recs, off = [], [], 0
    for i in range(count):
        inst = int(rng.integers(len(INSTANCES)))
        name = INSTANCES[inst][0]
        n = int(sizes[i])
        if name == "json":
            b = workloads.json(n, 1000 + i) if n else np.zeros(0, np.uint8)
        elif name == "log":
            b = workloads.loglines(n, int(rng.integers(5, 80))) if n else np.zeros(0, np.uint8)
        else:
            b = workloads.clike(n, 1000 + i, bcomment=name == "clike_b") if n else np.zeros(0, np.uint8)
        b = np.array(b, copy=True)
        if n > 2 and rng.random() < 0.1:  # a stray byte
            b[int(rng.integers(n))] = 1
        flags = 1 if rng.random() < 0.05 else 0
        parts.append(b)
        recs.append((off, n, inst, flags))
        off += n
    data = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    docs = np.array(recs, dtype=P.DOC_DTYPE)
    return data, docs


def check_batch(setup, data, docs, r):
    lexers, orcs, _ = setup
    assert r.status == 0
    kinds = r.kinds.cpu().numpy()
    lens = r.lens.cpu().numpy().view(np.uint32)
    offs = r.offsets.cpu().numpy() if r.offsets is not None else None
    nerr = 0
    total = 0
    for i, (doc, res) in enumerate(zip(docs, r.docs)):
        name, mode = INSTANCES[doc["inst"]]
        w = bytes(data[doc["offset"]: doc["offset"] + doc["length"]])
        k, l, o, con = orcs[name].lex(w, discard=bool(mode), offsets=True)
        assert res["status"] == 0
        assert res["error_offset"] == con, (i, name, res["error_offset"], con)
        assert res["ntokens"] == len(k), (i, name)
        assert res["tok_offset"] == total
        a, b = int(res["tok_offset"]), int(res["tok_offset"] + res["ntokens"])
        np.testing.assert_array_equal(kinds[a:b], k, err_msg=f"doc {i} ({name})")
        np.testing.assert_array_equal(lens[a:b], l, err_msg=f"doc {i} ({name})")
        if offs is not None:
            np.testing.assert_array_equal(offs[a:b], o.astype(np.int64), err_msg=f"doc {i} ({name})")
        total = b
        nerr += con < len(w)
    assert r.ntokens == total and r.nerrors == nerr


@pytest.mark.parametrize("lane", [16, 64, 1024, 4096])
def test_batch_mixed_instances(setup, lane):
    data, docs = make_docs(400, 7)
    print(f"[case] batch of {docs.size} docs, {data.size} B, lane {lane}", flush=True)
    _, _, batch = setup
    r = batch.run(torch.from_numpy(data).cuda(), docs, offsets=True, opts=P.RunOpts(lane_bytes=lane))
    check_batch(setup, data, docs, r)
    assert r.nslices > docs.size // 2


def test_batch_without_offsets_and_large_docs(setup):
    data, docs = make_docs(60, 8, median=64 << 10)
    _, _, batch = setup
    r = batch.run(torch.from_numpy(data).cuda(), docs, opts=P.RunOpts(lane_bytes=256))
    check_batch(setup, data, docs, r)


def test_batch_overflow_and_bad_table(setup):
    data, docs = make_docs(50, 9)
    _, _, batch = setup
    dev = torch.from_numpy(data).cuda()
    full = batch.run(dev, docs)
    r = batch.run(dev, docs, cap=full.ntokens - 1)
    assert r.status == P.LEX_EOVERFLOW and r.ntokens == full.ntokens
    assert (r.docs["status"] == P.LEX_EOVERFLOW).all()
    bad = docs.copy()
    bad[3]["length"] = data.size + 10  # outside the bytes: the planner rejects the table
    r = batch.run(dev, bad)
    assert r.status == P.LEX_EINVAL and (r.docs["status"] == P.LEX_EINVAL).all()
    bad = docs.copy()
    bad[5]["inst"] = len(INSTANCES)  # unknown instance
    r = batch.run(dev, bad)
    assert r.status == P.LEX_EINVAL


def test_batch_graph_replays(setup):
    """The launch sequence captured once and replayed, with eager work in between; every
    replay must equal the eager scan."""
    data, docs = make_docs(120, 10)
    _, _, batch = setup
    dev = torch.from_numpy(data).cuda()
    n, nd = data.size, docs.size
    docs_dev = torch.from_numpy(docs.view(np.uint8).copy()).cuda()
    kinds = torch.empty(n, dtype=torch.uint8, device="cuda")
    lens = torch.empty(n, dtype=torch.int32, device="cuda")
    res = torch.empty(nd * 32, dtype=torch.uint8, device="cuda")
    total = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(batch.workspace_size(nd, n), dtype=torch.uint8, device="cuda")
    eager = batch.run(dev, docs)
    want_k, want_l = eager.kinds.cpu().numpy(), eager.lens.cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run_into(dev, n, docs_dev, nd, kinds, lens, None, n, res, total, ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run_into(dev, n, docs_dev, nd, kinds, lens, None, n, res, total, ws,
                       stream=torch.cuda.current_stream())
    for rep in range(3):
        kinds.fill_(0xAA)
        lens.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        t = total.cpu().numpy()
        assert int(t[0]) == eager.ntokens, rep
        np.testing.assert_array_equal(kinds[: eager.ntokens].cpu().numpy(), want_k, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(lens[: eager.ntokens].cpu().numpy(), want_l, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(res[: nd * 32].cpu().numpy().view(P.DOC_RESULT_DTYPE), eager.docs)
        _ = batch.run(dev, docs)  # eager work between replays


SPEC_LANE = 2048  # a batch's speculative lane: the sync window, the shortest it allows


def test_batch_refused_hybrid_plan(setup):
    """Documents of the refused set C-like-B longer than one speculative lane (2 KiB) are
    split by the hybrid plan: each must still equal the oracle's serial scan, split clean
    documents report many slices, and those that must fall back (the serial scan halts; a
    block comment longer than the sync window across a lane boundary; a serial flag) run as
    one slice."""
    cb = INSTANCES.index(("clike_b", 1))
    parts, recs, off = [], [], 0

    def add(b, flags=0):
        nonlocal off
        b = np.array(b, dtype=np.uint8, copy=True)
        parts.append(b)
        recs.append((off, b.size, cb, flags))
        off += b.size

    for i, n in enumerate([4097, 5000, 8192, 300000, 1500000, 3000000]):
        add(workloads.clike(n, 900 + i, bcomment=True))
    bad = np.array(workloads.clike(200000, 910, bcomment=True), copy=True)
    bad[150000:150002] = ord("@")  # '@' is no token: the scan halts unless this lands in a comment or string
    add(bad)
    long_comment = np.concatenate([workloads.clike(3000, 911), np.frombuffer(b"\n/* " + b"x" * 5000 + b" */\n", np.uint8),
                                   workloads.clike(60000, 912)])
    add(long_comment)
    add(workloads.clike(100000, 913, bcomment=True), flags=1)
    # the last token (padding LFs: one whitespace token) spans the last lane's start
    add(np.concatenate([workloads.clike(8100, 914, bcomment=True), np.full(300, 10, np.uint8)]))
    data = np.concatenate(parts)
    docs = np.array(recs, dtype=P.DOC_DTYPE)
    print(f"[case] hybrid plan: {docs.size} C-like-B documents, {data.size} B", flush=True)
    _, _, batch = setup
    r = batch.run(torch.from_numpy(data).cuda(), docs, offsets=True)
    check_batch(setup, data, docs, r)
    ns = r.docs["nslices"]
    assert all(ns[i] > 1 for i in range(1, 6)), ns  # clean and longer than one lane: split
    assert ns[7] == 1 and ns[8] == 1, ns            # the long comment and the serial flag: one slice
    # the last lane empty: the previous one takes the rest (lanes of SPEC_LANE bytes)
    assert ns[9] == -(-8400 // SPEC_LANE) - 1, ns
    assert ns[5] >= 3000000 // 4096 // 2


@pytest.mark.parametrize("lane", [1024, 2048, 4096, 8192])
def test_batch_split_parts_at_batch_lanes(setup, lane):
    """The hybrid plan at the batch lanes the bench and the tuner use: a refused document
    longer than both the speculative lane (2 KiB) and the batch lane is split, and each slice
    is counted in four parts cut at serial token starts; the windowed emit adds the earlier
    parts' counts and starts a token at a window that begins a part.  Documents of many
    lengths (around 2, 4 and 8 KiB, and long ones), dense code and long (but shorter than the
    sync window) block comments near lane boundaries, with and without offsets: every
    document equals the oracle's serial scan, and those the plan splits report several
    slices."""
    cb = INSTANCES.index(("clike_b", 1))
    parts, recs, off = [], [], 0
    rng = np.random.default_rng(lane)
    lengths = [2047, 2048, 2049, 2100, 4095, 4096, 4097, 5000, 8191, 8193, 12000, 65536, 250000]
    for i, n in enumerate(lengths):
        b = np.array(workloads.clike(n, 2000 + i, bcomment=True), copy=True)
        parts.append(b)
        recs.append((off, n, cb, 0))
        off += n
    for i in range(6):  # comments of 300-1500 bytes starting just before 2 KiB boundaries
        b = bytearray()
        for k in range(1, 6):
            start = k * 2048 - int(rng.integers(50, 600))
            if len(b) < start:
                b += bytes(workloads.clike(start - len(b), 2100 + 10 * i + k))
            b += b"\n/* " + b"c" * int(rng.integers(300, 1500)) + b" */\n"
        b += bytes(workloads.clike(3000, 2190 + i))
        parts.append(np.frombuffer(bytes(b), np.uint8))
        recs.append((off, len(b), cb, 0))
        off += len(b)
    data = np.concatenate(parts)
    docs = np.array(recs, dtype=P.DOC_DTYPE)
    print(f"[case] split parts, batch lane {lane}: {docs.size} C-like-B documents, {data.size} B", flush=True)
    _, _, batch = setup
    opts = P.RunOpts(lane_bytes=lane)
    for offsets in (True, False):
        r = batch.run(torch.from_numpy(data).cuda(), docs, offsets=offsets, opts=opts)
        check_batch(setup, data, docs, r)
    ns = r.docs["nslices"]
    thr = max(2048, lane)
    for i, n in enumerate(lengths):
        if n > thr + 4096:
            assert ns[i] > 1, (i, n, ns[i])
        if n <= thr:
            assert ns[i] <= 1, (i, n, ns[i])  # one lane
