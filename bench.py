#!/usr/bin/env python3
"""Benchmark of the certified-split lexer on one MI355X.

A step is one scan of the whole hot path -- plan (certificate bitmap + cuts), count walk,
scan, emit walk -- over the 512 MiB C-like corpus in exact mode (token set C-like-L, lane
sub-chunks inside 64 KiB chunks), with the input already resident in HBM.  Prints one JSON
line: whole-job input GB/s, the roofline of the dominant kernel (HIP events around each
phase, on the scan's stream) and the oracle's single-core rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
MANIFEST_DIR = os.path.join(ROOT, "tests", "golden")  # the oracle's whole-stream digests
KERNEL_SOURCE = os.path.join(ROOT, "paper_2608_03473_amd", "csrc", "kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")  # *_hbm.md: counter summaries of the scan's kernels


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512 << 20, help="corpus bytes")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--lane-bytes", type=int, default=0)
    ap.add_argument("--chunk-bytes", type=int, default=64 << 10)
    ap.add_argument("--path", type=int, default=0, help="0 default, 1 pipeline, 2 fused, 3 one pass")
    ap.add_argument("--block-threads", type=int, default=0, help="threads per walk workgroup (0: default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle CPU time")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-documents leg")
    ap.add_argument("--batch-docs", type=int, default=50000)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-only", action="store_true",
                    help="batched leg without the per-document comparison (for kernel traces)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-framed", action="store_true", help="skip the framed-document leg")
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="per arrival rate (plus 1 s warm-up)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1 MiB, 256 MiB JSON and stray-byte configuration legs")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the library's default configuration instead of the autotuner's choice")
    ap.add_argument("--tune-cache", default=os.path.join("/tmp", "lexgpu_tune.json"))
    ap.add_argument("--only", choices=["framed"], default=None,
                    help="run that leg alone (no headline scan): for kernel traces and counters")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the chunked CPU baseline's all-cores figure (0: the cores this process may use)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one plain device copy of n bytes (scale for HBM counters)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from workloads import tokensets as T
    import paper_2608_03473_amd as P
    from paper_2608_03473_amd.hipevents import PhaseEvents

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    if args.only == "framed":
        print(json.dumps({"framed": framed_leg(args)}), flush=True)
        return
    t0 = time.time()
    host = workloads.clike(n, args.seed)
    log(args, f"corpus: {n} bytes in {time.time() - t0:.1f}s")
    data = torch.from_numpy(host).to(dev)
    lx = P.Lexer.compile(T.as_tuples(T.CLIKE_L))
    mode = P.LEX_MODE_EXACT
    opts = P.RunOpts(chunk_bytes=args.chunk_bytes, lane_bytes=args.lane_bytes, path=args.path,
                     block_threads=args.block_threads)
    tuning = None
    if not args.no_tune and not args.lane_bytes and not args.path and not args.block_threads:
        # the autotuner's configuration for this token set, mode, device and size (measured
        # here, every candidate checked against the defaults' output)
        from paper_2608_03473_amd import tune
        tu = tune.Tuner(cache_path=args.tune_cache)
        e = tu.tune(lx, data, mode, args.chunk_bytes, force=True)
        opts = tune.opts_of(e["opts"])
        tuning = {"choice": e["opts"], "plan": e["plan"], "ms": round(e["ms"], 4),
                  "default_ms": round(e["default_ms"], 4), "candidates": len(e["candidates"]),
                  "timing": "HIP events, median of 5 scans per candidate"}
        log(args, f"tuning: {tuning}")
        for c in sorted(e["candidates"], key=lambda c: c["ms"]):
            log(args, f"  candidate {c['ms']:.4f} ms {c['plan']} emit={c['opts'].get('emit', 0)}")
    cap = n
    kinds = torch.empty(cap, dtype=torch.uint8, device=dev)
    lens = torch.empty(cap, dtype=torch.int32, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = torch.empty(lx.workspace_size(n, mode, opts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_ref:
        # a plain shader copy (elementwise kernel: reads n bytes, writes n bytes), so the
        # HBM counters of the scan can be scaled by what they read for a known copy
        ref = torch.empty_like(data)
        torch.bitwise_or(data, 0, out=ref)
        torch.cuda.synchronize()
        del ref
    for _ in range(args.warmup):
        lx.run_into(data, n, mode, kinds, lens, None, cap, res, ws, opts)
    torch.cuda.synchronize()
    # the timed steps: the scan alone, as a caller runs it
    t_start = time.perf_counter()
    for k in range(args.steps):
        lx.run_into(data, n, mode, kinds, lens, None, cap, res, ws, opts, stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms = (t_end - t_start) * 1e3 / args.steps
    # the same steps again with HIP events at the phase boundaries (on the scan's stream),
    # for the per-kernel times and the roofline of the dominant kernel
    evs = [PhaseEvents() for _ in range(args.steps)]
    step_opts = []
    for e in evs:
        o = P.RunOpts(chunk_bytes=opts.chunk_bytes, lane_bytes=opts.lane_bytes, path=opts.path,
                      block_threads=opts.block_threads, emit=opts.emit)
        o.events = e.array
        step_opts.append(o)
    torch.cuda.synchronize()
    for k in range(args.steps):
        lx.run_into(data, n, mode, kinds, lens, None, cap, res, ws, step_opts[k], stream)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    ntok, err, status = int(r[0]), int(r[1]), int(np.int32(r[2] & 0xFFFFFFFF))
    nslices = int((int(r[2]) >> 32) & 0xFFFFFFFF)
    if status != 0 or err != n:
        print(f"bench: scan failed status={status} error_offset={err} n={n}", file=sys.stderr)
        sys.exit(1)
    parity = stream_parity("clike_512mib", n, args.seed, ntok, err, kinds, lens)
    phases = np.array([e.elapsed_ms() for e in evs])  # steps x 4
    ph_mean = phases.mean(axis=0)
    plan = lx.plan(n, mode, opts)
    if plan["path"] == 3:
        # one pass: reset, the one-pass kernel (plan, count walk, look-back, windowed emit),
        # scan, and the lane emit's fallback (it returns at once on a clean scan)
        names = ["reset", "onepass", "scan", "fallback_emit"]
        algo = {"reset": 0, "onepass": n + 5 * ntok, "scan": 0, "fallback_emit": 0}
    else:
        names = ["plan", "count_walk", "scan", "emit_walk"]
        algo = {"plan": n + n / 8, "count_walk": n, "scan": 0, "emit_walk": n + 5 * ntok}
    dom = names[int(np.argmax(ph_mean))]
    achieved = algo[dom] / (ph_mean[names.index(dom)] * 1e-3) / 1e9
    gbs = n / (ms * 1e-3) / 1e9
    path_bytes = n + 5 * ntok
    out = {
        "metric": "input GB/s lexed, 512 MiB",
        "value": round(gbs, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": f"C-like-L exact mode, {n} B C-like corpus (seed {args.seed}), "
                        f"{args.chunk_bytes} B chunks",
            "n_bytes": n, "tokens": ntok, "bytes_per_token": round(n / ntok, 3),
            "slices": nslices, "lane_bytes": plan["lane_bytes"], "path": plan["path"],
            "block_threads": plan["block_threads"],
        },
        "tokens_per_s": round(ntok / (ms * 1e-3), 1),
        "path_roofline_frac": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "parity": parity,
        "tuning": tuning,
        "phase_ms": {k: round(float(v), 4) for k, v in zip(names, ph_mean)},
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, n, plan),
            "algorithmic_bytes_per_launch": int(algo[dom]),
            "timing": "HIP events on the scan's stream at the phase boundaries, over a second pass of the "
                      "same steps right after the timed one (each event record adds about 3 us to a step)",
        },
        "cpu_baseline": None,
    }
    if not args.no_configs:
        out["configs"] = configs_leg(args, host, lx, kinds, lens, res)
    if not args.no_batched:
        del data, kinds, lens, ws
        torch.cuda.empty_cache()
        out["batched"] = batched_leg(args)
    if not args.no_framed:
        torch.cuda.empty_cache()
        out["framed"] = framed_leg(args)
    if not args.no_serving:
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host, args)
        out["cpu_chunked"] = cpu_chunked_leg(host, lx, args)
    print(json.dumps(out), flush=True)


def manifest_case(name):
    """The oracle's recorded digests for a benchmark case (tests/golden/stream_manifest.json,
    written from the oracle alone), or None."""
    try:
        with open(os.path.join(MANIFEST_DIR, "stream_manifest.json")) as f:
            return json.load(f)["cases"].get(name)
    except OSError:
        return None


def _digests(kinds_np, lens_np):
    sys.path.insert(0, MANIFEST_DIR)
    import stream_manifest as SM
    return SM.sha(kinds_np), SM.sha(lens_np.astype("<u4", copy=False))


def stream_parity(name, n, seed, ntok, err, kinds, lens):
    """Whole-stream parity of the last timed scan against the oracle's digests: token count,
    error offset, and the SHA-256 of every kind and every length.  None when the run is not
    the recorded workload."""
    case = manifest_case(name)
    if case is None or case.get("n") != n or case.get("seed") != seed:
        return None
    if ntok != case["ntokens"] or err != case["error_offset"]:
        return False
    k = kinds[:ntok].cpu().numpy()
    l = lens[:ntok].cpu().numpy().view("<u4")
    dk, dl = _digests(k, l)
    return dk == case["kinds"] and dl == case["lens"]


def timed_scan(lx, data, n, mode, kinds, lens, res, ws, opts, steps, warmup):
    """warmup untimed scans, then `steps` scans bracketed by synchronisations; ms per scan."""
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        lx.run_into(data, n, mode, kinds, lens, None, n, res, ws, opts, stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        lx.run_into(data, n, mode, kinds, lens, None, n, res, ws, opts, stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / steps


def configs_leg(args, host512, lx_l, kinds, lens, res):
    """The other single-buffer configurations, same protocol as the headline (input in HBM,
    outputs and workspace preallocated, warm-up then timed steps): the 1 MiB C-like corpus
    (seed 1, exact), the 512 MiB corpus with the stray 0x01 byte the oracle's rule picked
    (seed 3; the scan halts there, Corollary 1), and the 256 MiB JSON corpus in modulo-I
    mode (seed 4).  Each reports input GB/s, tokens/s, (N + 5 T_out) / t against 8 TB/s,
    the error offset and whole-stream parity with the oracle's digests."""
    import numpy as np
    import torch

    import workloads
    from workloads import tokensets as T
    import paper_2608_03473_amd as P

    dev = torch.device("cuda", 0)
    out = {}

    def leg(key, case_name, lx, buf, mode, steps, what):
        n = buf.size
        data = torch.from_numpy(buf).to(dev)
        opts = P.RunOpts(chunk_bytes=64 << 10)
        ws = torch.empty(lx.workspace_size(n, mode, opts), dtype=torch.uint8, device=dev)
        ms = timed_scan(lx, data, n, mode, kinds, lens, res, ws, opts, steps, args.warmup)
        r = res.cpu().numpy()
        ntok, err = int(r[0]), int(r[1])
        plan = lx.plan(n, mode, opts)
        case = manifest_case(case_name)
        par = None
        if case is not None:
            par = ntok == case["ntokens"] and err == case["error_offset"]
            if par:
                dk, dl = _digests(kinds[:ntok].cpu().numpy(), lens[:ntok].cpu().numpy().view("<u4"))
                par = dk == case["kinds"] and dl == case["lens"]
        out[key] = {
            "workload": what, "n_bytes": n, "ms": round(ms, 4), "steps": steps,
            "gbs": round(n / (ms * 1e-3) / 1e9, 3), "tokens": ntok, "tokens_per_s": round(ntok / (ms * 1e-3), 1),
            "roofline_frac": round((n + 5 * ntok) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "error_offset": err, "slices": int((int(r[2]) >> 32) & 0xFFFFFFFF),
            "path": plan["path"], "lane_bytes": plan["lane_bytes"], "parity": par,
        }
        log(args, f"config {key}: {out[key]}")
        del data, ws

    leg("config1_1mib", "clike_1mib", lx_l, workloads.clike(1 << 20, 1), P.LEX_MODE_EXACT, 200,
        "C-like-L exact mode, 1 MiB C-like corpus (seed 1), 64 KiB chunks (launch-bound)")
    stray = manifest_case("clike_512mib_stray_error")
    if stray is not None and host512.size == stray["n"] and args.seed == stray["seed"]:
        bad = np.array(host512, copy=True)
        bad[stray["stray_offset"]] = 1
        leg("config2_stray", "clike_512mib_stray_error", lx_l, bad, P.LEX_MODE_EXACT, args.steps,
            f"C-like-L exact mode, 512 MiB corpus (seed 2) with 0x01 at offset {stray['stray_offset']} "
            f"(seed 3, draw {stray['stray_draw']})")
        del bad
    lx_j = P.Lexer.compile(T.as_tuples(T.JSON))
    leg("config3_json", "json_256mib", lx_j, workloads.json(256 << 20, 4), P.LEX_MODE_DISCARD, args.steps,
        "JSON discard mode (WS deleted), 256 MiB pretty-printed JSON corpus (seed 4), 64 KiB chunks")
    torch.cuda.empty_cache()
    return out


def cpu_chunked_leg(host, lx, args):
    """The multithreaded chunked CPU lexer (lex_cpu_chunked, the paper's executor: 64 KiB
    equal-division chunks cut at certified bytes, threads taking chunks from a counter,
    ordered concatenation) over the library's packed table, on the same corpus in host
    memory: median of 5 passes at 1 thread, 8 threads and every core this process may use
    (no affinity mask).  A baseline for context, never a fallback of the GPU path."""
    import numpy as np

    n = host.size
    kinds = np.empty(n, np.uint8)
    lens = np.empty(n, np.uint32)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    allc = args.cpu_threads or max(1, min(avail, share))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    case = manifest_case("clike_512mib")
    out = {"kind": "multithreaded chunked lexer (lex_cpu_chunked)", "unit": "GB/s", "cpu_model": model,
           "nproc": os.cpu_count(), "cores_available": avail, "affinity_mask": False, "chunk_bytes": 64 << 10,
           "sample": f"the whole {n} B corpus in host memory, median of 5 passes"}
    for label, th in (("threads_1", 1), ("threads_8", 8), ("threads_all", allc)):
        ts = []
        for _ in range(5):
            t = time.perf_counter()
            k, l, nt, err, nch = lx.cpu_chunked(host, 0, chunk_bytes=64 << 10, threads=th, kinds=kinds, lens=lens)
            ts.append(time.perf_counter() - t)
        med = float(np.median(ts))
        par = None
        if case is not None and n == case["n"]:
            dk, dl = _digests(k, l)
            par = nt == case["ntokens"] and err == case["error_offset"] and dk == case["kinds"] and dl == case["lens"]
        out[label] = {"threads": th, "value": round(n / med / 1e9, 4), "ms": round(med * 1e3, 2),
                      "chunks": nch, "parity": par}
        log(args, f"cpu chunked {label}: {out[label]}")
    out["speedup_all_vs_1"] = round(out["threads_all"]["value"] / out["threads_1"]["value"], 2)
    return out


def batched_leg(args):
    """The batched-documents workload: 50,000 documents, log-normal sizes (median 16 KiB,
    sigma 1.5, 64 B - 8 MiB), C-like-L exact .475 / C-like-D discard .475 / C-like-B discard
    .05 (refused: one slice each).  One batched scan (lex_run_batch: one launch sequence,
    work-stealing tiles) against one lex_run per document, same library, same bytes in HBM,
    outputs and workspaces preallocated, on one stream and round-robin over four.  All must
    give the same token counts.  Also reported: the critical path, the largest refused
    document scanned alone."""
    import numpy as np
    import torch

    import workloads
    from workloads import tokensets as T
    import paper_2608_03473_amd as P

    t0 = time.time()
    buf, offs, sizes, sets = workloads.docs(args.batch_docs, 5)
    log(args, f"batched corpus: {args.batch_docs} docs, {buf.size} B in {time.time() - t0:.1f}s")
    insts = [(T.CLIKE_L, P.LEX_MODE_EXACT), (T.CLIKE_D, P.LEX_MODE_DISCARD), (T.CLIKE_B, P.LEX_MODE_DISCARD)]
    lexers = [P.Lexer.compile(T.as_tuples(d)) for d, _ in insts]
    batch = P.Batch([(lx, m) for lx, (_, m) in zip(lexers, insts)])
    dev = torch.device("cuda", 0)
    data = torch.from_numpy(buf).to(dev)
    n, nd = buf.size, args.batch_docs
    docs = np.zeros(nd, dtype=P.DOC_DTYPE)
    docs["offset"], docs["length"], docs["inst"] = offs, sizes, sets
    docs_dev = torch.from_numpy(docs.view(np.uint8).copy()).to(dev)
    bopts, btune = None, None
    if not args.no_tune:
        from paper_2608_03473_amd import tune
        tu = tune.Tuner(cache_path=args.tune_cache)
        e = tu.tune_batch(batch, [(lx, m) for lx, (_, m) in zip(lexers, insts)], data, docs_dev, nd, force=True)
        bopts = tune.opts_of(e["opts"])
        btune = {"choice": e["opts"], "ms": round(e["ms"], 3), "default_ms": round(e["default_ms"], 3),
                 "candidates": [(c["opts"].get("lane_bytes", 0), round(c["ms"], 3)) for c in e["candidates"]]}
        log(args, f"batch tuning: {btune}")
    kinds = torch.empty(n, dtype=torch.uint8, device=dev)
    lens = torch.empty(n, dtype=torch.int32, device=dev)
    res = torch.empty(nd * 32, dtype=torch.uint8, device=dev)
    total = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = torch.empty(batch.workspace_size(nd, n, bopts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        batch.run_into(data, n, docs_dev, nd, kinds, lens, None, n, res, total, ws, bopts, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_steps):
        batch.run_into(data, n, docs_dev, nd, kinds, lens, None, n, res, total, ws, bopts, stream=stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / args.batch_steps
    tot = total.cpu().numpy()
    ntok_batch = int(tot[0])
    per = res.cpu().numpy()[: nd * 32].view(P.DOC_RESULT_DTYPE)
    # parity of every document with the oracle's digests (counts, error offsets, tokens)
    case = manifest_case("docs_50k")
    par = None
    if case is not None and nd == case["count"]:
        sys.path.insert(0, MANIFEST_DIR)
        import stream_manifest as SM
        par = (SM.sha(per["ntokens"].astype("<u8")) == case["ntokens"]
               and SM.sha(per["error_offset"].astype("<u8")) == case["error_offsets"]
               and ntok_batch == case["total_tokens"])
        if par:
            dk, dl = _digests(kinds[:ntok_batch].cpu().numpy(), lens[:ntok_batch].cpu().numpy().view("<u4"))
            par = dk == case["kinds"] and dl == case["lens"]
    # the same launch sequence captured once in a hipGraph and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            batch.run_into(data, n, docs_dev, nd, kinds, lens, None, n, res, total, ws, bopts,
                           stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t) / args.batch_steps
    graph_same = int(total.cpu().numpy()[0]) == ntok_batch
    del g
    head = {
        "workload": f"{nd} documents, log-normal sizes (median 16 KiB, sigma 1.5, 64 B - 8 MiB), seed 5; "
                    "C-like-L exact / C-like-D discard / C-like-B discard (refused) = .475/.475/.05",
        "bytes": n, "tokens": ntok_batch,
        "batched_gbs": round(n / t_batch / 1e9, 3), "batched_ms": round(t_batch * 1e3, 3),
        "batched_graph_gbs": round(n / t_graph / 1e9, 3), "batched_graph_ms": round(t_graph * 1e3, 3),
        "graph_same_tokens": graph_same,
        "roofline_frac": round((n + 5 * ntok_batch) / min(t_batch, t_graph) / 1e9 / HBM_PEAK_GBS, 4),
        "parity": par,
        "tuning": btune,
        "workspace_mib": round(ws.numel() / 2**20, 1),
    }
    if args.batch_only:
        return head
    # one lex_run per document, back to back on the same stream
    cap = int(sizes.max())
    okinds = torch.empty(cap, dtype=torch.uint8, device=dev)
    olens = torch.empty(cap, dtype=torch.int32, device=dev)
    ores = torch.zeros((nd, 3), dtype=torch.int64, device=dev)
    wss = [torch.empty(lx.workspace_size(cap, m), dtype=torch.uint8, device=dev) for lx, (_, m) in zip(lexers, insts)]
    views = [data[int(o): int(o) + int(z)] for o, z in zip(offs, sizes)]

    def plain():
        for i in range(nd):
            k = int(sets[i])
            lexers[k].run_into(views[i], int(sizes[i]), insts[k][1], okinds, olens, None, cap, ores[i], wss[k], None,
                               stream)

    plain()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    ntok_plain = int(ores[:, 0].sum().item())
    same = ntok_plain == ntok_batch and bool((ores[:, 0].cpu().numpy() == per["ntokens"]).all())
    # the same per-document launches spread round-robin over four streams, each with its own
    # outputs and workspaces
    streams = [torch.cuda.Stream(device=dev) for _ in range(4)]
    sk = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in streams]
    sl = [torch.empty(cap, dtype=torch.int32, device=dev) for _ in streams]
    sws = [[torch.empty(lx.workspace_size(cap, m), dtype=torch.uint8, device=dev) for lx, (_, m) in zip(lexers, insts)]
           for _ in streams]
    ores4 = torch.zeros((nd, 3), dtype=torch.int64, device=dev)

    def plain4():
        for i in range(nd):
            k, q = int(sets[i]), i & 3
            lexers[k].run_into(views[i], int(sizes[i]), insts[k][1], sk[q], sl[q], None, cap, ores4[i], sws[q][k],
                               None, streams[q])

    torch.cuda.synchronize()
    plain4()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain4()
    torch.cuda.synchronize()
    t_plain4 = time.perf_counter() - t
    same = same and bool(torch.equal(ores4[:, 0], ores[:, 0]))
    # the critical path: the largest refused document, scanned alone (one lane)
    refused = np.flatnonzero(sets == workloads.DOC_B)
    crit = {}
    if refused.size:
        i = int(refused[np.argmax(sizes[refused])])
        k = int(sets[i])
        reps = 3
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            lexers[k].run_into(views[i], int(sizes[i]), insts[k][1], okinds, olens, None, cap, ores[i], wss[k], None,
                               stream)
        torch.cuda.synchronize()
        t_crit = (time.perf_counter() - t) / reps
        crit = {"critical_doc_bytes": int(sizes[i]), "critical_doc_ms": round(t_crit * 1e3, 3),
                "critical_doc_mbs": round(int(sizes[i]) / t_crit / 1e6, 1)}
    return {
        **head,
        "plain_gbs": round(n / t_plain / 1e9, 3), "plain_ms": round(t_plain * 1e3, 3),
        "speedup": round(t_plain / t_batch, 2),
        "plain_4streams_ms": round(t_plain4 * 1e3, 3), "speedup_vs_4streams": round(t_plain4 / t_batch, 2),
        "same_token_counts": same,
        "refused_docs": int((sets == workloads.DOC_B).sum()), **crit,
    }


def framed_leg(args):
    """Framing at the producer: a --n byte C-like-B document whose records (8 lines each)
    are opened by the reserved byte 0x1E, scanned in exact mode by the C-like-B set framed
    by that byte (lex_compile_framed: 0x1E certified, so the certified planner splits it),
    against the same-seed unframed document under the unframed set (refused: the hybrid
    plan).  Inputs resident in HBM, outputs and workspace preallocated, --steps timed scans
    after --warmup each."""
    import numpy as np
    import torch

    import workloads
    from workloads import tokensets as T
    import paper_2608_03473_amd as P

    dev = torch.device("cuda", 0)
    n, mode = args.n, P.LEX_MODE_EXACT
    defs = T.as_tuples(T.CLIKE_B)
    out = {"workload": f"C-like-B exact mode, {n} B C-like corpus with block comments (seed {args.seed}); "
                       "framed: records of 8 lines opened by 0x1E"}
    kinds = torch.empty(n, dtype=torch.uint8, device=dev)
    lens = torch.empty(n, dtype=torch.int32, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    for key, lx, frame in (("framed", P.Lexer.compile_framed(defs), 8), ("unframed", P.Lexer.compile(defs), 0)):
        host = workloads.clike(n, args.seed, bcomment=True, frame=frame)
        data = torch.from_numpy(host).to(dev)
        if args.copy_ref and frame:  # a plain copy of n bytes, to scale HBM counters
            ref = torch.empty_like(data)
            torch.bitwise_or(data, 0, out=ref)
            torch.cuda.synchronize()
            del ref
        ws = torch.empty(lx.workspace_size(n, mode), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            lx.run_into(data, n, mode, kinds, lens, None, n, res, ws, None, stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            lx.run_into(data, n, mode, kinds, lens, None, n, res, ws, None, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        r = res.cpu().numpy()
        plan = lx.plan(n, mode)
        par = stream_parity("clikeb_512mib_framed" if frame else "clikeb_512mib", n, args.seed, int(r[0]),
                            int(r[1]), kinds, lens)
        out[key] = {"gbs": round(n / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 3), "tokens": int(r[0]),
                    "error_offset": int(r[1]), "slices": int((int(r[2]) >> 32) & 0xFFFFFFFF),
                    "path": plan["path"], "hybrid": plan["hybrid"], "lane_bytes": plan["lane_bytes"],
                    "parity": par}
        if frame:
            out[key]["separators"] = int((host == 0x1E).sum())
        log(args, f"framed leg {key}: {out[key]}")
        del data, ws
    return out


def serving_leg(args):
    """The serving workload: open-loop Poisson arrivals at 2k, 10k and 50k requests/s,
    requests of log-normal size (median 8 KiB, sigma 1.5, 64 B - 4 MiB) drawn from a pool of
    3 x 2048 documents (C-like-L exact, C-like-D discard, JSON discard), 16 GiB HBM budget,
    four slots; p50/p99 latency from arrival to result in pinned host memory.  Each rate
    runs --serve-seconds after a 1 s warm-up (the paper-scale run is 60 s per rate:
    python -m paper_2608_03473_amd.serve)."""
    from paper_2608_03473_amd import serve

    pool = serve.make_pool(2048, 7)
    server = serve.Server(serve.instances(), budget_bytes=16 << 30, slots=4)
    out = {"seconds_per_rate": args.serve_seconds, "warmup_seconds": 1.0, "pool": "3 x 2048 documents",
           "deviation": "the configuration asks 60 s per rate; this bench runs --serve-seconds per rate to keep "
                        "the driver's run within minutes (the 60 s run: python -m paper_2608_03473_amd.serve "
                        "--seconds 60 --warmup 2 --pool 16384)",
           "rates": []}
    for rate in (2000.0, 10000.0, 50000.0):
        m = serve.open_loop(server, pool, rate, args.serve_seconds + 1.0, 6, warmup=1.0)
        log(args, f"serving {rate:.0f}/s: {m}")
        out["rates"].append(m)
    return out


def code_digest(path):
    """SHA-256 of a C/HIP source with its comments and whitespace removed: the counters of a
    kernel stay valid across edits of its comments, not across edits of its code."""
    import hashlib
    import re

    src = open(path, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()


def measured_traffic(kernel, n, plan):
    """HBM bytes per launch of the phase `kernel` from a committed rocprofv3 counter summary
    (profiles/*_hbm.md: FETCH_SIZE and WRITE_SIZE, scaled against a plain copy) taken on the
    same kernel code, workload size and resolved plan (path, lane length, workgroup size), or
    None when there is none."""
    import glob

    sha = code_digest(KERNEL_SOURCE)
    want = {"kernels_hip_code_sha256": sha, "workload_n": str(n), "path": str(plan["path"]),
            "lane_bytes": str(plan["lane_bytes"]), "block_threads": str(plan["block_threads"])}
    for path in sorted(glob.glob(os.path.join(PROFILES, "*_hbm.md"))):
        fields = {}
        try:
            with open(path, encoding="utf-8") as f:
                for line in f:
                    if ":" in line and not line.startswith(("|", "#", " ", "(")):
                        k, v = line.split(":", 1)
                        fields[k.strip()] = v.strip()
        except OSError:
            continue
        if all(fields.get(k) == v for k, v in want.items()):
            v = fields.get(f"traffic_bytes_{kernel}")
            return int(v) if v else None
    return None


def cpu_baseline(host, args):
    """The oracle (plain serial NFA lexer, single core) on a bounded prefix of the corpus."""
    import oracle
    from workloads import tokensets as T

    oc = oracle.OracleSet(T.as_tuples(T.CLIKE_L))
    probe = 4 << 20
    t = time.perf_counter()
    oc.lex(host[:probe])
    rate = probe / (time.perf_counter() - t)
    size = int(min(host.size, max(probe, rate * args.cpu_seconds)))
    t = time.perf_counter()
    k, _, con = oc.lex(host[:size])
    dt = time.perf_counter() - t
    log(args, f"oracle: {size} bytes, {len(k)} tokens in {dt:.1f}s")
    return {"value": round(size / dt / 1e9, 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {size} bytes of the same corpus ({len(k)} tokens, {dt:.1f} s)"}


if __name__ == "__main__":
    main()
