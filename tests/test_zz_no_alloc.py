"""lex_run_static, the scan entry point that allocates nothing, against lex_run.

Both run the same kernels; lex_run_static takes its workspace from the library's own
device scratch array instead of the caller's.  Each case makes two lex_run_static calls
in a row, the second on a smaller input (the scratch keeps the first call's contents),
and each must equal lex_run on the same input element by element: token count, error
offset, status, kinds, lengths and, where asked, offsets.  The cases cover the three
workspace layouts: the one-pass scan (C-like-L, exact), the fused scan with offsets (JSON,
modulo I) and the hybrid plan of a refused set (C-like-B).  A scan needing more workspace
than the scratch holds is refused on the host with LEX_ELIMIT before anything runs.
"""
import numpy as np
import pytest

import workloads
from workloads import tokensets as T

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2608_03473_amd")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _scan(lx, data, n, mode, static, offsets):
    dev = data.device
    cap = max(n, 1)
    # outputs prefilled with junk: neither entry point may depend on their contents
    kinds = torch.full((cap,), 0xEE, dtype=torch.uint8, device=dev)
    lens = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    offs = torch.full((cap,), -1, dtype=torch.int64, device=dev) if offsets else None
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    if static:
        lx.run_static_into(data, n, mode, kinds, lens, offs, cap, res)
    else:
        ws = torch.empty(lx.workspace_size(n, mode), dtype=torch.uint8, device=dev)
        lx.run_into(data, n, mode, kinds, lens, offs, cap, res, ws)
    r = res.cpu().numpy()
    ntok, err = int(r[0]), int(r[1])
    status = int(np.int32(r[2] & 0xFFFFFFFF))
    k = ntok if status == 0 else 0
    out = (kinds[:k].cpu().numpy(), lens[:k].cpu().numpy(), offs[:k].cpu().numpy() if offs is not None else None)
    return (ntok, err, status, int((int(r[2]) >> 32) & 0xFFFFFFFF)), out


CASES = [
    ("clike_l", lambda n, s: workloads.clike(n, s), P.LEX_MODE_EXACT, False, (24 << 20) + 77, (1 << 20) + 5),
    ("json", lambda n, s: workloads.json(n, s), P.LEX_MODE_DISCARD, True, (16 << 20) + 3, 300001),
    ("clike_b", lambda n, s: workloads.clike(n, s, bcomment=True), P.LEX_MODE_DISCARD, False, 8 << 20, 300017),
]


@pytest.mark.parametrize("name,gen,mode,offsets,n1,n2", CASES, ids=[c[0] for c in CASES])
def test_static_equals_lex_run_twice(name, gen, mode, offsets, n1, n2):
    lx = P.Lexer.compile(T.as_tuples(T.NAMED[name]))
    for call, n in enumerate((n1, n2)):
        assert lx.workspace_size(n, mode) <= P.abi.LEX_STATIC_WS_BYTES
        buf = gen(n, 40 + call)
        data = torch.from_numpy(buf).cuda()
        print(f"[case] lex_run_static {name} mode={mode} n={n} call {call}", flush=True)
        got_meta, got = _scan(lx, data, n, mode, True, offsets)
        want_meta, want = _scan(lx, data, n, mode, False, offsets)
        assert got_meta == want_meta, (name, call)
        assert want_meta[2] == 0 and want_meta[1] == n, (name, call)
        for g, w in zip(got, want):
            if w is not None:
                np.testing.assert_array_equal(g, w, err_msg=f"{name} call {call}")


def test_static_refuses_oversized_scan():
    """A scan needing more than the scratch holds is refused on the host (nothing runs)."""
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    n = 300 << 20
    assert lx.workspace_size(n, P.LEX_MODE_EXACT) > P.abi.LEX_STATIC_WS_BYTES
    data = torch.zeros(n, dtype=torch.uint8, device="cuda")
    kinds = torch.empty(n, dtype=torch.uint8, device="cuda")
    lens = torch.empty(n, dtype=torch.int32, device="cuda")
    res = torch.zeros(3, dtype=torch.int64, device="cuda")
    with pytest.raises(P.LexError) as e:
        lx.run_static_into(data, n, P.LEX_MODE_EXACT, kinds, lens, None, n, res)
    assert e.value.code == P.LEX_ELIMIT
