"""Benchmark of the epsilon-cost sharded VFilter on one MI355X.

Workload (one step = the whole hot path): build a VFilter with b = 8 over
n = 2^27 distinct synthetic uint64 keys with h = 11 (2048 shards of about
2^16 keys, eps = 0.0175 in eq. (logballsbins)), then answer 2^30 queries
(half members drawn with replacement, half fresh non-members).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "build Mkeys/s + query Gq/s (VFilter b=8, 2^27 keys); serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch (per query pass for the grouped query, whose kernels
# run once per chunk) of this workload measured with rocprofv3 PMC counters
# (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy); see
# profiles/vfilter_b8_n2p27_hbm_traffic_pmc.md.  They hold for the kernel
# source with this SHA-256 prefix only and are reported as null otherwise.
PMC_SOURCE_SHA = "f28f41b75e3f6698"
PMC_TRAFFIC_BYTES = {"k_build": 94.04e9, "k_query": 410.88e9, "query_grouped": 58.16e9,
                     "k_scatter": 2.97e9, "k_count+k_scan": 1.09e9}


def pmc_traffic(kernel: str):
    import hashlib
    src = os.path.join(ROOT, "paper_2503_18397_amd", "csrc", "vf_device.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return PMC_TRAFFIC_BYTES.get(kernel) if sha == PMC_SOURCE_SHA else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--log2n", type=int, default=27)
    p.add_argument("--log2q", type=int, default=30)
    p.add_argument("--b", type=int, default=8)
    p.add_argument("--eps", type=float, default=0.0175)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--data-seed", type=int, default=2027)
    p.add_argument("--sigma", type=int, default=None, help="override lg segment size")
    p.add_argument("--query", choices=("grouped", "plain"), default="grouped",
                   help="grouped: queries grouped by shard first (vfilter_contains_grouped, "
                        "its workspace is the build's); plain: one gather per probe")
    p.add_argument("--group-chunk-log2", type=int, default=None,
                   help="grouped queries: chunks of 2^k keys (default: the library's largest)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-packed", action="store_true",
                   help="batch workload: cells of 1/2/4/8 bytes instead of b-bit fields")
    p.add_argument("--no-batch", action="store_true",
                   help="leave the batched workload out of the default line")
    p.add_argument("--no-serve", action="store_true",
                   help="skip the short serving trace measured after the timed region")
    p.add_argument("--line-serve-builds", type=int, default=24,
                   help="builds of the serving trace reported in the default line")
    p.add_argument("--cpu-sample-shards", type=int, default=16)
    p.add_argument("--workload", choices=("vfilter", "batch", "serve", "stream", "mwhc"),
                   default="vfilter",
                   help="vfilter: the sharded VFilter (default); batch: 100 000 independent "
                        "VFuncs of 10..50 000 keys in one launch per cell width, against "
                        "one build per instance; serve: a Poisson stream of builds and "
                        "query batches served with --slots slots against one request at a time")
    p.add_argument("--stream-log2n", type=int, default=32,
                   help="stream: keys (in pinned host memory) of the VFilter")
    p.add_argument("--stream-chunk-log2", type=int, default=28)
    p.add_argument("--stream-query", choices=("plain", "grouped"), default="plain",
                   help="query path of the streamed workload (grouping does not pay "
                        "with 2^16 shards: every chunk loads every shard's cells)")
    p.add_argument("--slots", type=int, default=4)
    p.add_argument("--serve-builds", type=int, default=48)
    p.add_argument("--serve-queries", type=int, default=480)
    p.add_argument("--batch-count", type=int, default=100000)
    p.add_argument("--batch-sample", type=int, default=300,
                   help="instances built one by one for the per-instance comparison")
    return p.parse_args()


def stream_main(args) -> None:
    """One GPU's share of a multi-GPU build: a VFilter (b = 8) over 2^32
    keys held in pinned host memory, copied in 2^28-key chunks while
    earlier chunks are counted by shard, 2^16 shards of about 2^16 keys,
    then 2^32 mixed queries (50% members) against the HBM-resident
    structure."""
    import torch
    import synthetic as S
    import paper_2503_18397_amd as vf

    dev = torch.device("cuda:0")
    n, chunk = 1 << args.stream_log2n, 1 << args.stream_chunk_log2
    h = max(0, args.stream_log2n - 16)
    print(f"[bench] stream: 2^{args.stream_log2n} keys in pinned host memory", file=sys.stderr,
          flush=True)
    keys = torch.empty(n, dtype=torch.int64, pin_memory=True)
    for c0 in range(0, n, chunk):
        cnt = min(chunk, n - c0)
        i = torch.arange(c0, c0 + cnt, dtype=torch.int64, device=dev)
        keys[c0:c0 + cnt].copy_(S.feistel(2 * i, args.data_seed))
    opts = vf.vf_default_opts(h=h)
    sz = vf.vf_plan(n, args.b, 0.0, True, opts)
    ws = torch.empty(sz.workspace_bytes + (8 * n + 255) // 256 * 256, dtype=torch.uint8,
                     device=dev)
    st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
    Q = n
    torch.cuda.synchronize()
    print("[bench] stream: build", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    rc, hd = vf.vfilter_build_host(keys, args.b, 0.0, args.seed, opts, ws, st, chunk, stream)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = vf.vf_info(hd)
    print(f"[bench] stream: build {build_s:.3f} s, rc {rc}; queries", file=sys.stderr,
          flush=True)
    # queries in chunks (generated on the device), timed with events; the
    # grouped path uses the build's workspace, free once the build returned
    qms, fp, neg, members_ok = 0.0, 0, 0, True
    out = torch.empty(chunk, dtype=torch.uint8, device=dev)
    grouped = args.stream_query == "grouped"
    if grouped:
        gws = ws[: vf.vf_query_grouped_bytes(hd, chunk)]
    for c0 in range(0, Q, chunk):
        cnt = min(chunk, Q - c0)
        q, is_mem = S.queries_chunk(n, c0, cnt, args.data_seed, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if grouped:
            vf.vfilter_contains_grouped(hd, q, out[:cnt], gws, stream)
        else:
            vf.vfilter_contains(hd, q, out[:cnt], stream)
        e1.record(stream)
        e1.synchronize()
        qms += e0.elapsed_time(e1)
        o = out[:cnt]
        members_ok = members_ok and bool(o[is_mem].min().item() == 1)
        fp += int(o[~is_mem].sum().item())
        neg += int((~is_mem).sum().item())
        del q, is_mem
    vf.vf_free(hd)
    res = {
        "metric": "streamed build Mkeys/s + query Gq/s (VFilter b=8, keys from pinned host)",
        "value": round(n / build_s / 1e6, 3), "unit": "Mkeys/s",
        "query": {"value": round(Q / (qms * 1e-3) / 1e9, 4), "unit": "Gq/s",
                  "path": args.stream_query},
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"VFilter b={args.b}, n=2^{args.stream_log2n} keys streamed from "
                               f"pinned host in 2^{args.stream_chunk_log2}-key chunks, h={h}, "
                               f"2^{args.stream_log2n} queries (50% members)",
                   "n": n, "h": info["h"], "M": info["M"], "sigma": info["sigma"],
                   "V": info["V"]},
        "build_s_with_transfer": round(build_s, 3),
        "device_phases_ms": {"copy+count+scan": round(info["ms_count"], 3),
                             "scatter": round(info["ms_scatter"], 3),
                             "k_build": round(info["ms_build"], 3)},
        "pcie_gbs": round(8 * n / (info["ms_count"] * 1e-3) / 1e9, 2),
        "check": {"rc": rc, "members_all_true": members_ok, "fpr_x256":
                  round(256 * fp / max(neg, 1), 4), "failed_attempts": info["n_failures"],
                  "relaunched_shards": info["relaunched_shards"],
                  "space_bits_per_key": round(info["space_bits"] / n, 4)},
    }
    print(json.dumps(res), flush=True)


def serve_measure(args, builds: int, queries: int) -> dict:
    """Serving loop: builds (10^3..10^7 keys, b in {4,8,16}, VFunc:VFilter
    1:1) and query batches (1..10^6 keys, 90% members) arriving as Poisson
    streams, served with --slots slots and again one request at a time; the
    same trace both times, structures resident in HBM (200 GB budget); then
    the whole trace submitted at once (saturated) both ways.  The served runs
    merge waiting query batches into combined launches (vf_query_multi); one
    request at a time does not."""
    import torch
    import synthetic as S
    from paper_2503_18397_amd.serve import Request, Server, poisson_trace

    dev = torch.device("cuda:0")
    ev = poisson_trace(args.data_seed + 4, builds, queries, build_rate=40.0, query_rate=400.0)
    data = {}
    for e in ev:
        if e["kind"] != "query":
            data[e["id"]] = (S.member_keys(e["n"], 300 + e["id"], device=dev),
                             S.values(e["n"], e["b"], 300 + e["id"], device=dev))
    for j, e in enumerate(ev):
        if e["kind"] == "query":
            e["keys"], _ = S.queries(data[e["target"]][0], e["n"], 700 + j,
                                     member_share_per_256=230)
    torch.cuda.synchronize()
    print(f"[bench] serve: {builds} builds, {queries} query batches",
          file=sys.stderr, flush=True)

    def serve(slots, paced=True, coalesce=16):
        srv = Server(slots=slots, coalesce=coalesce)
        t0 = time.perf_counter()
        for j, e in enumerate(ev):
            while paced and time.perf_counter() - t0 < e["t"]:
                time.sleep(0.0002)
            if e["kind"] == "query":
                srv.submit(Request(10000 + j, "query", e["keys"], target=e["target"]))
            else:
                k, v = data[e["id"]]
                srv.submit(Request(e["id"], e["kind"], k, v, b=e["b"], eps=args.eps))
        st = srv.drain(timeout=600)
        srv.close()
        out = st.summary()
        out["merged_query_launches"] = srv.merged_launches
        return out

    serve(args.slots)  # warm-up (allocator, kernels)
    mixed = serve(args.slots)
    print(f"[bench] served: {mixed}", file=sys.stderr, flush=True)
    one = serve(1, coalesce=1)
    print(f"[bench] one at a time: {one}", file=sys.stderr, flush=True)
    # saturated: the whole trace at once, so the device and not the
    # arrivals bounds the throughput
    sat = serve(args.slots, paced=False)
    sat1 = serve(1, paced=False, coalesce=1)
    print(f"[bench] saturated: {sat} / one at a time {sat1}", file=sys.stderr, flush=True)

    def kps(x):
        return (x["build"]["keys"] + x["query"]["keys"]) / x["makespan_s"]

    return {
        "workload": f"{builds} builds (10^3..10^7 keys, b in {{4,8,16}}, VFunc:VFilter 1:1) "
                    f"at 40/s, {queries} query batches (1..10^6 keys, 90% members) at 400/s, "
                    "200 GB HBM budget",
        "slots": args.slots,
        "build_p50_ms": mixed["build"]["p50_ms"], "build_p99_ms": mixed["build"]["p99_ms"],
        "query_p50_ms": mixed["query"]["p50_ms"], "query_p99_ms": mixed["query"]["p99_ms"],
        "served": mixed, "one_at_a_time": one,
        "saturated": {"served": sat, "one_at_a_time": sat1,
                      "keys_per_s": round(kps(sat), 1),
                      "one_at_a_time_keys_per_s": round(kps(sat1), 1),
                      "speedup_keys_per_s": round(kps(sat) / kps(sat1), 3)},
    }


def serve_main(args) -> None:
    r = serve_measure(args, args.serve_builds, args.serve_queries)
    mixed = r["served"]
    res = {
        "metric": "serve p50/p99 ms and keys/s (Poisson builds and query batches)",
        "value": mixed.get("build", {}).get("keys_per_s"), "unit": "built keys/s",
        "higher_is_better": True, "n_gpus": 1, "vs_baseline": None, "data": "synthetic",
        "config": {"workload": r["workload"], "slots": args.slots},
        "served": mixed, "one_at_a_time": r["one_at_a_time"], "saturated": r["saturated"],
    }
    print(json.dumps(res), flush=True)


def batch_main(args) -> None:
    print(json.dumps(batch_measure(args)), flush=True)


def batch_measure(args) -> dict:
    """Batched uneven instances: one build launch per cell width for all
    instances (vf_batch_build) against one vf_build per instance, timed on
    a random sample of the same instances."""
    import numpy as np
    import torch
    import synthetic as S
    import paper_2503_18397_amd as vf

    dev = torch.device("cuda:0")
    n, b = S.batch_shape(args.batch_count, args.data_seed + 2)
    total = int(n.sum())
    print(f"[bench] batch: {n.size} instances, {total} keys", file=sys.stderr, flush=True)
    keys = S.member_keys(total, args.data_seed + 2, device=dev)
    vals = S.batch_values(n, b, args.data_seed + 2, device=dev)
    inst = torch.repeat_interleave(torch.arange(n.size, dtype=torch.int32, device=dev),
                                   torch.as_tensor(n.astype(np.int64), device=dev))
    out = torch.empty(total, dtype=torch.int64, device=dev)
    # cells packed to b bits each (bit-array storage), unless --no-packed
    opts = vf.vf_default_opts(packed=0 if args.no_packed else 1)
    sz = vf.vf_batch_plan(n, b, opts)
    ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
    st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        rc, h = vf.vf_batch_build(keys, vals, n, b, args.seed, opts, ws, st, stream)
        e[1].record(stream)
        vf.vf_batch_query(h, inst, keys, out, stream)
        e[2].record(stream)
        e[2].synchronize()
        info = vf.vf_info(h)
        res = (rc, e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), info)
        vf.vf_free(h)
        return res

    for i in range(args.warmup):
        step()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(step())
        print(f"[bench] batch step {i}: build {recs[-1][1]:.3f} ms, query {recs[-1][2]:.3f} ms",
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    rc, _, _, info = recs[-1]
    build_ms = sum(r[1] for r in recs) / len(recs)
    query_ms = sum(r[2] for r in recs) / len(recs)
    bits = torch.as_tensor(b.astype(np.int64), device=dev)[inst.long()]
    ok = bool(torch.equal(out, vals & ((torch.ones_like(bits) << bits) - 1)))

    # one build per instance (vf_build with h = 0), buffers allocated once
    rng = np.random.default_rng(args.data_seed)
    sample = rng.choice(n.size, min(args.batch_sample, n.size), replace=False)
    off = np.concatenate([[0], np.cumsum(n.astype(np.int64))])
    o1 = vf.vf_default_opts(h=0)
    big = max(vf.vf_plan(int(n[i]), int(b[i]), 0.0, False, o1).workspace_bytes for i in sample)
    bst = max(vf.vf_plan(int(n[i]), int(b[i]), 0.0, False, o1).structure_bytes for i in sample)
    ws1 = torch.empty(big, dtype=torch.uint8, device=dev)
    st1 = torch.empty(bst, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    keys_done = 0
    for i in sample:
        k = keys[off[i]:off[i + 1]]
        v = vals[off[i]:off[i + 1]]
        rc1, h1 = vf.vf_build(k, v, int(b[i]), 0.0, args.seed, o1, ws1, st1, stream)
        vf.vf_free(h1)
        keys_done += int(n[i])
    torch.cuda.synchronize()
    per_s = time.perf_counter() - t1
    batched = total / (build_ms * 1e-3) / 1e6
    single = keys_done / per_s / 1e6
    res = {
        "metric": "batched build Mkeys/s (independent VFuncs, one launch per cell width)",
        "value": round(batched, 3), "unit": "Mkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "build_ms": round(build_ms, 3), "query_ms": round(query_ms, 3),
        "query": {"value": round(total / (query_ms * 1e-3) / 1e9, 4), "unit": "Gq/s"},
        "higher_is_better": True, "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{n.size} VFuncs, sizes log-uniform in [10, 50000], "
                               "b uniform in {1,4,8,16,32}, h = 0 each",
                   "instances": int(n.size), "keys": total},
        "check": {"rc": rc, "all_members_answer_their_value": ok,
                  "failed_instances": info["failed_shards"],
                  "failed_attempts": info["n_failures"],
                  "relaunched_instances": info["relaunched_shards"],
                  "space_bits_per_key": round(info["space_bits"] / total, 4),
                  "stored_bits_per_key": round(8 * sz.structure_bytes / total, 4),
                  "mean_b": round(float((n.astype(np.float64) * b).sum() / total), 4),
                  "packed": not args.no_packed},
        "per_instance_launches": {"value": round(single, 3), "unit": "Mkeys/s",
                                  "instances_timed": int(sample.size), "keys": keys_done,
                                  "seconds": round(per_s, 3)},
        "speedup_vs_per_instance": round(batched / single, 2),
    }
    del keys, vals, inst, out, ws, st, ws1, st1
    torch.cuda.empty_cache()
    return res


def cpu_baseline(args, keys_np=None, queries_np=None) -> dict:
    """The oracle on the GPU machine's host cores: the whole build of the same
    workload (every shard; shards split over host threads, the C oracle
    running with the interpreter lock released) and a sample of 2^24 of the
    same queries in chunks over the same threads; for context, one thread on
    16 shards of the same shape and 2^21 queries."""
    import concurrent.futures as cf
    import numpy as np
    import oracle as O
    import synthetic as S
    mwhc = args.workload == "mwhc"
    threads = max(1, min(16, os.cpu_count() or 1))
    n = 1 << args.log2n
    if keys_np is None:
        keys_np = S.member_keys(n, args.data_seed).numpy().view(np.uint64)
    h = O.shard_bits_eps(n, args.eps)
    t0 = time.perf_counter()
    built = O.build_threaded(keys_np, b=args.b, is_filter=True, h=h, seed=args.seed,
                             threads=threads, mwhc=mwhc)
    t1 = time.perf_counter()
    qs = queries_np[: 1 << 24] if queries_np is not None else \
        S.queries(S.member_keys(n, args.data_seed), 1 << 24, args.data_seed)[0].numpy().view(
            np.uint64)
    with cf.ThreadPoolExecutor(threads) as ex:
        t2 = time.perf_counter()
        list(ex.map(lambda c: O.query(built, c), np.array_split(qs, threads)))
        t3 = time.perf_counter()
    del built
    # one thread, 16 shards of about 2^16 keys
    n_s = args.cpu_sample_shards << 16
    h_s = (args.cpu_sample_shards - 1).bit_length()
    k1 = S.member_keys(n_s, args.data_seed)
    q1, _ = S.queries(k1, 1 << 21, args.data_seed)
    t4 = time.perf_counter()
    b1 = O.build(k1.numpy().view(np.uint64), b=args.b, is_filter=True, h=h_s, seed=args.seed,
                 mwhc=mwhc)
    t5 = time.perf_counter()
    O.query(b1, q1.numpy().view(np.uint64))
    t6 = time.perf_counter()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": round(n / (t1 - t0) / 1e6, 4),
        "unit": "Mkeys/s",
        "query_value": round(qs.size / (t3 - t2) / 1e9, 6),
        "query_unit": "Gq/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole build (n={n}, h={h}, b={args.b}, {1 << h} shards) on {threads} "
                  f"threads; {qs.size} of the same queries",
        "nproc": os.cpu_count(), "cpu": model,
        "single_thread": {"value": round(n_s / (t5 - t4) / 1e6, 4), "unit": "Mkeys/s",
                          "query_value": round(q1.numel() / (t6 - t5) / 1e9, 6),
                          "query_unit": "Gq/s", "cores": 1,
                          "sample": f"{args.cpu_sample_shards} shards x ~2^16 keys "
                                    f"(n={n_s}, h={h_s}); 2^21 mixed queries"},
    }


def copy_bandwidth(torch, dev) -> float:
    """Device-to-device copy of 2 GiB (reads 2 GiB, writes 2 GiB), best of
    five, in GB/s: the measured ceiling beside the 8 TB/s specification."""
    x = torch.empty(1 << 28, dtype=torch.int64, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(5):
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    torch.cuda.empty_cache()
    return 2 * 2.0 ** 31 / (best * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        batch_main(args)
        return
    if args.workload == "serve":
        serve_main(args)
        return
    if args.workload == "stream":
        stream_main(args)
        return
    mwhc = args.workload == "mwhc"
    if mwhc and args.eps == 0.0175:
        args.eps = 0.01  # section 4.1 sets epsilon = 0.01 for MWHC
    import torch
    import synthetic as S
    import paper_2503_18397_amd as vf

    dev = torch.device("cuda:0")
    n, Q = 1 << args.log2n, 1 << args.log2q
    print(f"[bench] generating n=2^{args.log2n} keys, 2^{args.log2q} queries on {dev}",
          file=sys.stderr, flush=True)
    keys = S.member_keys(n, args.data_seed, device=dev)
    queries, is_member = S.queries(keys, Q, args.data_seed)
    n_neg = int((~is_member).sum().item())
    out = torch.empty(Q, dtype=torch.uint8, device=dev)
    opts = vf.vf_default_opts(sigma=args.sigma, mwhc=int(mwhc))
    sz = vf.vf_plan(n, args.b, args.eps, True, opts)
    ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
    st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    copy_gbs = copy_bandwidth(torch, dev)
    qws = ws if args.group_chunk_log2 is None else None

    def step(timed: bool):
        nonlocal qws
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        rc, h = vf.vfilter_build(keys, args.b, args.eps, args.seed, opts, ws, st, stream)
        if qws is None:
            qws = ws[:vf.vf_query_grouped_bytes(h, 1 << args.group_chunk_log2)]
        e[1].record(stream)
        if args.query == "grouped":
            # the build's workspace is free once vfilter_build has returned
            vf.vfilter_contains_grouped(h, queries, out, qws, stream)
        else:
            vf.vfilter_contains(h, queries, out, stream)
        e[2].record(stream)
        e[2].synchronize()
        info = vf.vf_info(h)
        res = (rc, e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), info)
        vf.vf_free(h)
        return res

    for i in range(args.warmup):
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        recs.append(step(True))
        print(f"[bench] step {i}: build {recs[-1][1]:.3f} ms, query {recs[-1][2]:.3f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    rc, _, _, info = recs[-1]
    members_ok = bool(out[is_member].min().item() == 1)
    fp = int(out[~is_member].sum().item())
    build_ms = sum(r[1] for r in recs) / len(recs)
    query_ms = sum(r[2] for r in recs) / len(recs)
    k_build_ms = sum(r[3]["ms_build"] for r in recs) / len(recs)
    k_count_ms = sum(r[3]["ms_count"] for r in recs) / len(recs)
    k_scatter_ms = sum(r[3]["ms_scatter"] for r in recs) / len(recs)
    S_, V, cb = info["S"], info["V"], info["cell_bytes"]

    # algorithmic bytes per launch (measurement)
    kern = {
        "k_build": {"ms": k_build_ms, "bytes": 8 * n + S_ * V * cb + S_},
        "k_query": {"ms": query_ms, "bytes": Q * (8 + 3 * cb + 1), "path": args.query},
        "k_count+k_scan": {"ms": k_count_ms, "bytes": 8 * n},
        "k_scatter": {"ms": k_scatter_ms, "bytes": 8 * n + 8 * n},
    }
    for name, k in kern.items():
        k["traffic"] = None if mwhc else pmc_traffic(
            "query_grouped" if name == "k_query" and args.query == "grouped" else name)
        k["GB/s"] = round(k["bytes"] / (k["ms"] * 1e-3) / 1e9, 2) if k["ms"] > 0 else None
        k["frac"] = round(k["GB/s"] / HBM_PEAK_GBS, 5) if k["GB/s"] else None
    # The build's algorithmic bytes per key: read the key, write it grouped
    # by shard, read it back, write the structure (cells and local seeds).
    # k_build is the build's dominant kernel (its launch is almost all of
    # the build's time), so the build's bytes are priced on its duration.
    build_bpk = 8 + 8 + 8 + (S_ * V * cb + S_) / n
    build_gbs = build_bpk * n / (k_build_ms * 1e-3) / 1e9
    query_gbs = kern["k_query"]["GB/s"]
    res = {
        "metric": METRIC,
        "value": round(n / (build_ms * 1e-3) / 1e6, 3),
        "unit": "Mkeys/s",
        "query": {"value": round(Q / (query_ms * 1e-3) / 1e9, 4), "unit": "Gq/s"},
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "build_ms": round(build_ms, 3),
        "query_ms": round(query_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": (f"VFilter b={args.b}, n=2^{args.log2n} uint64 keys, "
                                f"{'MWHC 3-partite hypergraphs' if mwhc else 'fuse graphs'}, "
                                f"eps={args.eps} (h={info['h']}, {info['S']} shards of "
                                f"~{n // max(info['S'], 1)} keys), 2^{args.log2q} queries "
                                "(50% members)"),
                   "n": n, "queries": Q, "b": args.b, "eps": args.eps, "h": info["h"],
                   "M": info["M"], "sigma": info["sigma"], "l": info["l"], "V": V,
                   "c": f"{info['c_num']}/{info['c_den']}", "query_path": args.query,
                   "parallelism": "1 GPU"},
        "check": {"rc": rc, "members_all_true": members_ok, "negatives": n_neg,
                  "false_positives": fp, "fpr_x256": round(256 * fp / max(n_neg, 1), 4),
                  "failed_attempts": info["n_failures"],
                  "relaunched_shards": info["relaunched_shards"],
                  "space_bits_per_key": round(info["space_bits"] / n, 4)},
        "roofline": {"bound": "hbm", "kernel": "k_build", "achieved": round(build_gbs, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(build_gbs / HBM_PEAK_GBS, 5),
                     "traffic": kern["k_build"]["traffic"],
                     "bytes_per_key": round(build_bpk, 3),
                     "basis": "the build's algorithmic bytes (read key, write and read it "
                              "grouped by shard, write cells and seeds) per k_build launch",
                     "k_build_own": {"bytes_per_key": round(kern["k_build"]["bytes"] / n, 3),
                                     "achieved": kern["k_build"]["GB/s"],
                                     "frac": kern["k_build"]["frac"]},
                     "query": {"bytes_per_query": 8 + 3 * cb + 1, "achieved": query_gbs,
                               "frac": kern["k_query"]["frac"], "path": args.query},
                     "copy_GBps": round(copy_gbs, 1),
                     "frac_of_copy": round(build_gbs / copy_gbs, 5)},
        "kernels": kern,
    }
    del ws, st
    if not args.no_serve and not mwhc:
        # the serving loop, measured after the timed region
        res["serve"] = serve_measure(args, args.line_serve_builds, 10 * args.line_serve_builds)
    if not args.no_batch and not mwhc:
        # the batched workload (--workload batch), one timed step, after the
        # timed region
        import copy
        bargs = copy.copy(args)
        bargs.steps, bargs.warmup = 1, 1
        res["batch"] = batch_measure(bargs)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on host cores)", file=sys.stderr, flush=True)
        import numpy as np
        k_np = keys.cpu().numpy().view(np.uint64)
        q_np = queries[: 1 << 24].cpu().numpy().view(np.uint64)
        res["cpu_baseline"] = cpu_baseline(args, k_np, q_np)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
