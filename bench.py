"""Benchmark: elements/s and HBM GB/s versus region length, tag versus signal.

Workload: 2^26 hash-generated u32 elements in fixed-length regions, enumerated,
filtered (bit 0 of H(x,0)), expanded into 0..3 children and aggregated per region
(count, u64 sum, min, max).  A step is one pass of the whole path over the batch:
the reset kernel and one launch of the persistent pipeline kernel, with the inputs
already resident in HBM.  The headline's steps are graph replays (`run_again` replays
the captured reset + pipeline kernels, as a caller's does), HIP events around all of
them.  The sweep's steps, and the headline's `direct_launches` figure, are direct
launches: those pipelines are created with RS_TIME_KERNEL, which brackets every
pipeline kernel with a HIP event pair (the kernel durations of the roofline) and
therefore launches directly instead of replaying a graph.  Three copies of the input
rotate between steps so that the 256 MB last-level cache does not serve the reads.

Prints one JSON line: the headline at L = 4096, the sweep over
L in {1, 4, 16, 64, 256, 1024, 4096} for every strategy, the roofline of the
pipeline kernel, and the serial oracle timed on a bounded sample on the host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_ELEMENTS = 1 << 26
LENGTHS = [1, 4, 16, 64, 256, 1024, 4096]
HEADLINE_L = 4096
HBM_PEAK_GBS = 8000.0
STRATEGY_NAMES = {0: "tag", 1: "signal", 3: "lanes", 4: "enum+tag"}
COPIES = 3


KERNEL_SOURCE = os.path.join(ROOT, "paper_2006_07478_amd", "csrc", "rs_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hash_expand_L4096.json")


def kernel_source_hash():
    """Hash of the pipeline kernel's device code: the file up to its host-side launch table,
    with line comments and whitespace dropped, so that a change to host code or to comments
    alone keeps counter summaries valid."""
    with open(KERNEL_SOURCE, "rb") as f:
        src = f.read().decode()
    cut = src.find("// ---------------------------------------------------------------- launch table")
    if cut >= 0:
        src = src[:cut]
    code = " ".join(line.split("//", 1)[0].strip() for line in src.splitlines())
    return hashlib.sha256(" ".join(code.split()).encode()).hexdigest()[:16]


def measured_traffic(strategy, width):
    """HBM bytes per launch from the committed counter summary, if it was taken on this
    kernel source for this configuration; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            entries = json.load(f).get("entries", [])
    except (OSError, ValueError, AttributeError):
        return None
    src = kernel_source_hash()
    for t in entries:
        if (t.get("kernel_source_sha256_16") == src and t.get("strategy") == strategy
                and t.get("ensemble_width") == width):
            return t.get("hbm_bytes_per_launch")
    return None


def parse_widths(arg):
    """--width: one ensemble width for every strategy ("256"; 0 lets the autotuner choose) or one
    per strategy ("tag:128,signal:64,lanes:64,enum_tag:128").  Returns {strategy name: width}."""
    names = ("tag", "signal", "lanes", "enum_tag")
    if ":" not in arg:
        return {n: int(arg) for n in names}
    out = {n: 0 for n in names}
    for kv in arg.split(","):
        k, v = kv.split(":")
        if k.strip() not in out:
            raise ValueError(f"unknown strategy {k!r} in --width")
        out[k.strip()] = int(v)
    return out


def algorithmic_bytes(n, L):
    """Bytes the path must move per run: elements, CSR offsets, 20 B of aggregates per region."""
    R = (n + L - 1) // L
    return 4 * n + 4 * (R + 1) + 20 * R


def time_config(rs, torch, stream, offsets, copies, strategy, width, steps, warmup, stats=False):
    """Time `steps` launches rotating over the input copies.  Returns ms per step (HIP events on
    the launch stream around the whole timed region: reset + pipeline kernels and any gaps), the
    pipeline kernel's own mean duration (event pairs the library records around it on the same
    stream, RS_TIME_KERNEL), the ensemble width and the statistics."""
    pipes = []
    for vals in copies:
        p = rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width,
                        flags=rs.RS_TIME_KERNEL | (rs.RS_COLLECT_STATS if stats else 0))
        p.set_stream(stream.cuda_stream)
        sid = p.push(offsets, vals, n_elements=N_ELEMENTS)   # device tensors: borrowed, already in HBM
        p.run()
        pipes.append((p, sid))
    st0 = pipes[0][0].stats(pipes[0][1])
    chosen, qdepth = int(st0.ensemble_width), int(st0.queue_depth)
    for i in range(warmup):
        pipes[i % len(pipes)][0].run_again(rs.RS_RUN_ASYNC)
    torch.cuda.synchronize()
    for p, _ in pipes:
        p.kernel_times()   # drop the untimed launches
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        pipes[i % len(pipes)][0].run_again(rs.RS_RUN_ASYNC)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kt = [t for p, _ in pipes for t in p.kernel_times()]
    assert len(kt) == steps, (len(kt), steps)
    kernel_ms = {"mean": sum(kt) / len(kt), "median": float(np.median(kt)), "min": min(kt), "queue_depth": qdepth}
    st = pipes[0][0].stats(pipes[0][1]) if stats else None
    for p, _ in pipes:
        p.close()
    return ms, kernel_ms, chosen, st


def time_graph_replay(rs, torch, stream, offsets, copies, strategy, width, steps, warmup):
    """The same steps as time_config, replayed from each pipeline's captured HIP graph (reset and
    pipeline kernels): ms per step from events around all of them."""
    pipes = []
    for vals in copies:
        p = rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width)
        p.set_stream(stream.cuda_stream)
        p.push(offsets, vals, n_elements=N_ELEMENTS)
        p.run()
        pipes.append(p)
    for i in range(warmup):
        pipes[i % len(pipes)].run_again(rs.RS_RUN_ASYNC)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        pipes[i % len(pipes)].run_again(rs.RS_RUN_ASYNC)
    e1.record(stream)
    torch.cuda.synchronize()
    for p in pipes:
        p.close()
    return e0.elapsed_time(e1) / steps


def occupancy_pass(rs, torch, stream, offsets, vals, strategy, width, L):
    """One launch with device statistics (kept out of the timed launches): lane occupancy and share
    of full firings per node; for signals beside the closed form L/(w ceil(L/w)) of the
    enumerating node (§5)."""
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width, flags=rs.RS_COLLECT_STATS) as p:
        p.set_stream(stream.cuda_stream)
        sid = p.push(offsets, vals, n_elements=N_ELEMENTS)
        p.run()
        st = p.stats(sid)
    occ = lambda k: round(st.items[k] / max(1, st.firings[k] * width), 4)
    full = lambda k: round(st.full[k] / max(1, st.firings[k]), 4)
    out = {"enum_occupancy": occ(0), "enum_full_frac": full(0), "expand_occupancy": occ(1),
           "agg_occupancy": occ(2), "agg_full_frac": full(2)}
    if strategy in (rs.RS_SIGNAL, rs.RS_ENUM_TAG) and L > 0:
        out["enum_occupancy_closed_form"] = round(L / (width * -(-L // width)), 4)
    return out


VARIABLE_MAX = [2, 8, 32, 128, 512, 2048, 8192]


def variable_sweep(rs, torch, stream, copies, steps, warmup, width=0):
    """Region sizes uniform in [0, max] over 2^26 elements, both strategies (the paper's second
    synthetic experiment): elements/s and algorithmic GB/s from the pipeline kernel's mean, and
    the enumerating node's lane occupancy beside its closed form sum(n) / (w sum(ceil(n/w)))."""
    import workloads
    rows = []
    for mx in VARIABLE_MAX:
        offs_h = workloads.variable_offsets(2, N_ELEMENTS, mx)
        sizes = np.diff(offs_h.astype(np.int64))
        R = len(sizes)
        offsets = torch.from_numpy(offs_h.view(np.int32)).cuda()
        row = {"max": mx, "regions": R}
        for s, name in ((rs.RS_TAG, "tag"), (rs.RS_SIGNAL, "signal"), (rs.RS_SIGNAL_LANES, "lanes"),
                        (rs.RS_ENUM_TAG, "enum+tag")):
            ms, kt, w, _ = time_config(rs, torch, stream, offsets, copies, s, width, steps, warmup)
            kms = kt["mean"]
            nbytes = 4 * N_ELEMENTS + 4 * (R + 1) + 20 * R
            row[name] = {"ensemble_width": w, "queue_depth": kt["queue_depth"], "ms": round(ms, 4),
                         "kernel_ms": round(kms, 4),
                         "elements_per_s": N_ELEMENTS / (kms * 1e-3), "GB_per_s": round(nbytes / (kms * 1e-3) / 1e9, 1)}
            occ = occupancy_pass(rs, torch, stream, offsets, copies[0], s, w, 0)
            row[name]["enum_occupancy"] = occ["enum_occupancy"]
            if s in (rs.RS_SIGNAL, rs.RS_ENUM_TAG):
                row[name]["enum_occupancy_closed_form"] = round(float(sizes.sum()) / (w * float(np.sum(-(-sizes // w)))), 4)
            print(f"[bench] variable max={mx:5d} {name:8s} w={w:4d} kernel {kms:8.3f} ms  "
                  f"{N_ELEMENTS / (kms * 1e-3) / 1e9:7.2f} Gelem/s", file=sys.stderr, flush=True)
        rows.append(row)
    return rows


def output_stream_rate(rs, torch, stream, vals, L, steps=5):
    """The ordered output stream (emit_outputs) at the headline size, both strategies: the
    pipeline kernel's median, and algorithmic bytes with 4 B per output item added."""
    offsets = torch.from_numpy(__import__("workloads").fixed_offsets(N_ELEMENTS, L).view(np.int32)).cuda()
    res = {}
    for s, name in ((rs.RS_TAG, "tag"), (rs.RS_SIGNAL, "signal"), (rs.RS_SIGNAL_LANES, "lanes")):
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=s, ensemble_width=0, emit_outputs=True,
                         flags=rs.RS_TIME_KERNEL) as p:
            p.set_stream(stream.cuda_stream)
            sid = p.push(offsets, vals, n_elements=N_ELEMENTS)
            p.run()
            st = p.stats(sid)
            for _ in range(2):
                p.run_again(rs.RS_RUN_ASYNC)
            torch.cuda.synchronize()
            p.kernel_times()
            for _ in range(steps):
                p.run_again(rs.RS_RUN_ASYNC)
            kt = p.kernel_times()
        ms = float(np.median(kt))
        nbytes = algorithmic_bytes(N_ELEMENTS, L) + 4 * int(st.n_outputs)
        res[name] = {"ensemble_width": int(st.ensemble_width), "n_outputs": int(st.n_outputs),
                     "kernel_ms_median": round(ms, 4), "elements_per_s": N_ELEMENTS / (ms * 1e-3),
                     "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    return res


def probe_copy(rs, torch, stream, nbytes=1 << 30, reps=10):
    """The library's plain 1 GiB copy: achievable-bandwidth reference and counter calibration."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(2):
        rs.hbm_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        rs.hbm_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes": 2 * nbytes, "ms": round(ms, 4), "GB_per_s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def serving(rs, torch, stream, n_streams=512, rhos=(0.5, 0.8, 1.2), headline_rho=0.8, arrival_seeds=(6, 7, 8),
            budget=2 << 30):
    """512 streams of the serving workload (log-uniform sizes 1e3..1e7, log-uniform mean region
    length 1..4096, hash/expand pipeline).

    gpu: all streams resident in HBM, one batched persistent launch versus one launch per stream
         on the same HIP stream (replayed, event-timed).
    serve: the native request loop on host-memory requests under an HBM budget; capacity is
         measured with every request arriving at once, then requests arrive as a Poisson process
         at rho times that capacity (rho 0.5, 0.8, 1.2; three arrival seeds each); latency is
         completion minus arrival (host clock), p50/p99 over all requests of the three seeds.
    """
    import workloads
    n, m = workloads.stream_shapes(seed=5, n_streams=n_streams)
    reqs = [workloads.serving_stream(5, s, int(n[s]), float(m[s])) for s in range(n_streams)]
    total = int(n.sum())
    out = {"streams": n_streams, "elements": total, "hbm_budget_bytes": budget,
           "requests": "host memory, pinned (page-locked), as a serving front end would receive them"}

    # --- GPU side: batched persistent launch vs one launch per stream
    dev = [(torch.from_numpy(o.view(np.int32)).cuda(), torch.from_numpy(v.view(np.int32)).cuda()) for o, v in reqs]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_AUTO, ensemble_width=0, flags=rs.RS_COLLECT_STATS) as p:
        p.set_stream(stream.cuda_stream)
        ids = [p.push(o, v, n_elements=len(v)) for o, v in dev]
        p.run()
        st = p.stats(ids[0])
        strategy, width = int(st.strategy), int(st.ensemble_width)
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width) as p:
        p.set_stream(stream.cuda_stream)
        for o, v in dev:
            p.push(o, v, n_elements=len(v))
        p.run()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            p.run_again(rs.RS_RUN_ASYNC)
        e1.record(stream)
        torch.cuda.synchronize()
        batched_ms = e0.elapsed_time(e1) / 5
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width) as p:
        p.set_stream(stream.cuda_stream)
        for rep in range(2):   # the first pass warms up
            for o, v in dev:
                p.push(o, v, n_elements=len(v))
            torch.cuda.synchronize()
            e0.record(stream)
            p.run(rs.RS_RUN_PER_STREAM | rs.RS_RUN_ASYNC)
            e1.record(stream)
            torch.cuda.synchronize()
            per_stream_ms = e0.elapsed_time(e1)
    out["gpu"] = {"strategy": STRATEGY_NAMES.get(strategy, str(strategy)), "ensemble_width": width,
                  "batched_ms": round(batched_ms, 3), "batched_elements_per_s": total / (batched_ms * 1e-3),
                  "per_stream_ms": round(per_stream_ms, 3),
                  "per_stream_elements_per_s": total / (per_stream_ms * 1e-3)}

    # --- end to end: the request loop on host-memory requests, held in pinned buffers (filled
    # before any timing) so the host-to-device copies run at DMA speed
    def pinned(a):
        t = torch.empty(len(a), dtype=torch.int32, pin_memory=True)
        t.numpy()[:] = a.view(np.int32)
        return t.numpy().view(np.uint32)

    reqs = [(pinned(o), pinned(v)) for o, v in reqs]

    def run_serve(arrival_sets, per_stream, requests=None, device_out=None):
        lat, rates, launches = [], [], 0
        for arrivals in arrival_sets:
            with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=width,
                             hbm_budget_bytes=budget) as p:
                _, tim = p.serve(reqs if requests is None else requests, arrivals, per_stream=per_stream,
                                 device_out=device_out)
            lat += [t["completed"] - t["arrival"] for t in tim]
            span = max(t["completed"] for t in tim) - min(t["arrival"] for t in tim)
            rates.append(total / span)
            launches += len({t["batch"] for t in tim})
        lat = np.array(lat)
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "elements_per_s": float(np.mean(rates)), "launches": launches, "requests": len(lat)}

    sat = run_serve([np.zeros(n_streams)], False)
    capacity = sat["elements_per_s"]
    by_rho = {}
    for rho in rhos:
        rate = rho * capacity / (total / n_streams)
        sets = [workloads.arrivals(seed, n_streams, rate) for seed in arrival_seeds]
        by_rho[str(rho)] = {"arrival_rate_per_s": rate, "batched": run_serve(sets, False),
                            "per_stream": run_serve(sets, True)}
        print(f"[bench] serve rho={rho}: {json.dumps(by_rho[str(rho)])}", file=sys.stderr, flush=True)
    head = by_rho[str(headline_rho)]
    out["serve"] = {"capacity_elements_per_s": capacity, "rho": headline_rho, "arrival_seeds": list(arrival_seeds),
                    "arrival_rate_per_s": head["arrival_rate_per_s"], "batched": head["batched"],
                    "per_stream": head["per_stream"], "by_rho": by_rho}
    # the same loop on requests already resident in HBM whose aggregates the kernel writes into
    # device arrays of the caller: no copies over the link either way, so it shows what the loop
    # and the GPU sustain
    douts = [{"count": torch.empty(max(len(o) - 1, 1), dtype=torch.int32, device="cuda"),
              "sum": torch.empty(max(len(o) - 1, 1), dtype=torch.int64, device="cuda"),
              "min": torch.empty(max(len(o) - 1, 1), dtype=torch.int32, device="cuda"),
              "max": torch.empty(max(len(o) - 1, 1), dtype=torch.int32, device="cuda")} for o, _ in reqs]
    run_serve([np.zeros(n_streams)], False, requests=dev, device_out=douts)   # warm-up
    sat_d = run_serve([np.zeros(n_streams)], False, requests=dev, device_out=douts)
    cap_d = sat_d["elements_per_s"]
    rate_d = headline_rho * cap_d / (total / n_streams)
    sets_d = [workloads.arrivals(seed, n_streams, rate_d) for seed in arrival_seeds]
    out["serve_device"] = {"requests": "device memory (resident in HBM), aggregates written into device arrays",
                           "capacity_elements_per_s": cap_d,
                           "capacity_vs_batched_gpu": cap_d / out["gpu"]["batched_elements_per_s"],
                           "saturation_launches": sat_d["launches"],
                           "rho": headline_rho, "arrival_rate_per_s": rate_d,
                           "batched": run_serve(sets_d, False, requests=dev, device_out=douts),
                           "per_stream": run_serve(sets_d, True, requests=dev, device_out=douts)}
    del douts
    print(f"[bench] serve device-resident: {json.dumps(out['serve_device'])}", file=sys.stderr, flush=True)
    del dev
    return out


def other_configs(rs, torch, stream, steps=5):
    """The other workloads beside the hash/expand sweep, each at its full size, both strategies,
    widths from the autotuner: C1 (4096 parents of 0..64 u32, mod-4 filter; latency-bound, so the
    replay latency of one launch is reported), C3 (1 GiB of text lines: words and longest word per
    line; elements are bytes) and C4 (2^24 vertices, 2^28 weighted edges, per-vertex threshold
    filter; count and sum)."""
    import workloads

    def dev(a):
        a = np.ascontiguousarray(a)
        return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).cuda()

    def kernel_rate(kind, offsets, elements, n_bytes_alg, lengths=None, parent_param=None, fields=None, param=None):
        res = {}
        strats = ((rs.RS_TAG, "tag"), (rs.RS_SIGNAL, "signal"))
        if kind != rs.RS_TEXT_WORDS:
            strats += ((rs.RS_SIGNAL_LANES, "lanes"),)
        if kind in (rs.RS_TEXT_WORDS, rs.RS_HASH_EXPAND, rs.RS_HASH_TREE):
            strats += ((rs.RS_ENUM_TAG, "enum+tag"),)
        for s, name in strats:
            kw = {} if param is None else {"param": param}
            with rs.Pipeline(kind, strategy=s, ensemble_width=0, agg_fields=fields, flags=rs.RS_TIME_KERNEL,
                             **kw) as p:
                p.set_stream(stream.cuda_stream)
                sid = p.push(offsets, elements, lengths=lengths, parent_param=parent_param,
                             n_elements=int(elements.numel()))
                p.run()
                st = p.stats(sid)
                w, q = int(st.ensemble_width), int(st.queue_depth)
                for _ in range(2):
                    p.run_again(rs.RS_RUN_ASYNC)
                torch.cuda.synchronize()
                p.kernel_times()
                for _ in range(steps):
                    p.run_again(rs.RS_RUN_ASYNC)
                kt = p.kernel_times()
            ms = float(np.median(kt))
            n = int(elements.numel())
            res[name] = {"ensemble_width": w, "queue_depth": q, "kernel_ms_median": round(ms, 4),
                         "elements_per_s": n / (ms * 1e-3), "GB_per_s": round(n_bytes_alg / (ms * 1e-3) / 1e9, 1)}
        return res

    out = {}
    # C1: replay latency of one launch (graph replay), events around each replay
    offsets, vals = workloads.modfilter_workload(seed=1)
    o, v = dev(offsets), dev(vals)
    c1 = {}
    for s, name in ((rs.RS_TAG, "tag"), (rs.RS_SIGNAL, "signal"), (rs.RS_SIGNAL_LANES, "lanes")):
        with rs.Pipeline(rs.RS_MODFILTER, strategy=s, ensemble_width=0, agg_fields=rs.RS_COUNT | rs.RS_SUM,
                         param=(4, 0, 0, 0)) as p:
            p.set_stream(stream.cuda_stream)
            sid = p.push(o, v, n_elements=len(vals))
            p.run()
            w = int(p.stats(sid).ensemble_width)
            lat = []
            for r in range(23):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                p.run_again(rs.RS_RUN_ASYNC)
                e1.record(stream)
                torch.cuda.synchronize()
                if r >= 3:
                    lat.append(e0.elapsed_time(e1) * 1e3)
        c1[name] = {"ensemble_width": w, "replay_us_median": round(float(np.median(lat)), 1),
                    "replay_us_min": round(float(np.min(lat)), 1)}
    out["C1_modfilter_4096_parents"] = {"n_elements": len(vals), "n_parents": len(offsets) - 1, **c1}
    # C3: 1 GiB of text
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 30)
    R = len(starts)
    out["C3_text_1GiB"] = {"n_elements": len(text), "n_parents": R, **kernel_rate(
        rs.RS_TEXT_WORDS, dev(starts), dev(text), len(text) + 8 * R + 8 * R, lengths=dev(lengths),
        fields=rs.RS_COUNT | rs.RS_MAX)}
    del text, starts, lengths
    # the taxi-shaped text (long lines of mean 1397 bytes, few spaces): the three versions of the
    # paper's taxi comparison are signals, enumeration then tags, and tags
    text, starts, lengths = workloads.taxi_workload(seed=9, total_bytes=1 << 30)
    R = len(starts)
    out["taxi_text_1GiB"] = {"n_elements": len(text), "n_parents": R, **kernel_rate(
        rs.RS_TEXT_WORDS, dev(starts), dev(text), len(text) + 8 * R + 8 * R, lengths=dev(lengths),
        fields=rs.RS_COUNT | rs.RS_MAX)}
    del text, starts, lengths
    # tree topology: the filter feeds the expansion and a second aggregating node (kept count
    # and sum) at the headline size, regions of 16 and 4096
    vals = workloads.hash_values(2, N_ELEMENTS)
    dv = dev(vals)
    for L in (16, 4096):
        offsets = workloads.fixed_offsets(N_ELEMENTS, L)
        R = len(offsets) - 1
        out[f"tree_2p26_L{L}"] = {"n_elements": N_ELEMENTS, "n_parents": R, **kernel_rate(
            rs.RS_HASH_TREE, dev(offsets), dv, 4 * N_ELEMENTS + 4 * (R + 1) + 32 * R,
            fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE])}
    del vals, dv
    # C4: 2^24 vertices, 2^28 edges
    offsets, w, thr, _ = workloads.graph_workload(seed=4)
    R = len(offsets) - 1
    N = len(w)
    out["C4_graph_2p28_edges"] = {"n_elements": N, "n_parents": R, **kernel_rate(
        rs.RS_GRAPH_THRESH, dev(offsets), dev(w), 4 * N + 4 * (R + 1) + 4 * R + 12 * R, parent_param=dev(thr),
        fields=rs.RS_COUNT | rs.RS_SUM)}
    return out


def host_info():
    """CPU model and thread counts of the machine the bench runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"host_cpu": model, "host_logical_cpus": os.cpu_count(), "host_usable_cpus": usable}


def cpu_baseline(L, budget_s=12.0):
    """The serial oracle on a bounded sample of the same workload (single thread)."""
    import oracle
    import workloads
    n = 1 << 22
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while True:
        oracle.run(oracle.HASH_EXPAND, offsets, vals)
        reps += 1
        t = time.perf_counter() - t0
        if t >= budget_s or reps >= 512:
            break
    out = {"value": reps * n / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
           "sample": f"{reps} runs of 2^22 elements (regions of {L}) of the same generator, "
                     f"single-threaded serial oracle, {t:.1f} s"}
    out.update(host_info())
    return out


def cpu_baseline_threads(L, budget_s=6.0):
    """The same serial oracle function on T contiguous parent ranges at once (one thread each,
    T = the job's CPU share); the concatenated records must equal the serial run's."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import workloads
    n = 1 << 24
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    # the job's CPU share: OMP_NUM_THREADS where the host sets it, never more than 16 threads
    T = max(1, min(host_info()["host_usable_cpus"], int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 16))
    P = len(offsets) - 1
    cuts = [P * i // T for i in range(T + 1)]
    parts = [(offsets[a:b + 1] - offsets[a], vals[offsets[a]:offsets[b]]) for a, b in zip(cuts, cuts[1:])]
    run_part = lambda ov: oracle.run(oracle.HASH_EXPAND, ov[0], ov[1])
    with ThreadPoolExecutor(T) as pool:
        got = list(pool.map(run_part, parts))
        ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
        for f in ("count", "sum", "min", "max"):
            if not np.array_equal(np.concatenate([getattr(g, f) for g in got]), getattr(ref, f)):
                raise AssertionError(f"threaded oracle differs from the serial run in {f}")
        reps, t0 = 0, time.perf_counter()
        while True:
            list(pool.map(run_part, parts))
            reps += 1
            t = time.perf_counter() - t0
            if t >= budget_s or reps >= 256:
                break
    return {"value": reps * n / t, "unit": "elements/s", "cores": T, "kind": "oracle",
            "sample": f"{reps} runs of 2^24 elements (regions of {L}), the serial oracle on {T} contiguous "
                      f"parent ranges in {T} threads, results checked equal to one serial run, {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--width", default="0",
                    help="ensemble width (0 lets the autotuner choose), or one per strategy as tag:128,signal:64")
    ap.add_argument("--headline-only", action="store_true", help="time only L = 4096 (for profiling)")
    ap.add_argument("--lengths", default="",
                    help="comma-separated region lengths to time instead of the whole sweep (for profiling); "
                         "prints the sweep rows only unless 4096 is among them")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing of the headline")
    ap.add_argument("--configs-only", action="store_true",
                    help="time only the other workloads (C1, C3, taxi-shaped text, tree, C4), for profiling")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--strategy", choices=["tag", "signal", "lanes", "enum_tag", "both", "all"], default="all",
                    help="lanes: the lane-resolved signals the paper proposes as future work; enum_tag: "
                         "enumeration in the first stage, tags after it")
    ap.add_argument("--no-occupancy", action="store_true", help="skip the per-node statistics pass of the sweep")
    ap.add_argument("--no-serving", action="store_true", help="skip the 512-stream batching/serving leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1/C3/C4 workloads")
    ap.add_argument("--no-variable", action="store_true", help="skip the variable-size sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library runs on a single MI355X and has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("RS_AUTOTUNE_CACHE", "/tmp/regionstream-autotune-bench.txt")
    import torch
    import paper_2006_07478_amd as rs
    import workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.configs_only:
        print(json.dumps({"configs": other_configs(rs, torch, stream)}))
        return
    t_gen = time.perf_counter()
    # three resident copies (seeds 2, 102, 202); the first is the seed-2 workload
    copies = [torch.from_numpy(workloads.hash_values(2 + 100 * c, N_ELEMENTS).view(np.int32)).cuda()
              for c in range(COPIES)]
    print(f"[bench] generated {COPIES} x 2^26 elements in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
    strategies = {"tag": [rs.RS_TAG], "signal": [rs.RS_SIGNAL], "lanes": [rs.RS_SIGNAL_LANES],
                  "enum_tag": [rs.RS_ENUM_TAG], "both": [rs.RS_TAG, rs.RS_SIGNAL],
                  "all": [rs.RS_TAG, rs.RS_SIGNAL, rs.RS_SIGNAL_LANES, rs.RS_ENUM_TAG]}[args.strategy]
    names = {rs.RS_TAG: "tag", rs.RS_SIGNAL: "signal", rs.RS_SIGNAL_LANES: "lanes", rs.RS_ENUM_TAG: "enum+tag"}
    lengths = [HEADLINE_L] if args.headline_only else LENGTHS
    partial = bool(args.lengths)
    if partial:
        lengths = [int(x) for x in args.lengths.split(",")]
    width_of = lambda s: parse_widths(args.width).get(names[s].replace("+", "_"), 0)
    sweep = []
    head = {}
    for L in lengths:
        offsets = torch.from_numpy(workloads.fixed_offsets(N_ELEMENTS, L).view(np.int32)).cuda()
        row = {"L": L}
        for s in strategies:
            ms, kt, w, _ = time_config(rs, torch, stream, offsets, copies, s, width_of(s), args.steps,
                                       args.warmup)
            kms = kt["mean"]
            eps = N_ELEMENTS / (ms * 1e-3)
            gbs = algorithmic_bytes(N_ELEMENTS, L) / (ms * 1e-3) / 1e9
            row[names[s]] = {"ms": round(ms, 4), "kernel_ms": round(kms, 4), "elements_per_s": eps,
                             "GB_per_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "ensemble_width": w,
                             "queue_depth": kt["queue_depth"]}
            if not args.no_occupancy and not args.headline_only and not partial:   # the profiled commands
                row[names[s]].update(occupancy_pass(rs, torch, stream, offsets, copies[0], s, w, L))
            print(f"[bench] L={L:5d} {names[s]:8s} w={w:4d} {ms:8.3f} ms  {eps / 1e9:7.2f} Gelem/s  {gbs:7.1f} GB/s",
                  file=sys.stderr, flush=True)
            if L == HEADLINE_L:
                head[names[s]] = (ms, eps, gbs, w, kt)
        sweep.append(row)

    if partial and not head:
        print(json.dumps({"sweep": sweep, "n_elements": N_ELEMENTS, "steps": args.steps, "warmup": args.warmup}))
        return
    best = max(head, key=lambda k: head[k][1])
    ms, eps, gbs, w_best, kt_best = head[best]
    best_s = {v: k for k, v in names.items()}[best]
    graph_ms = None
    if not args.no_graph:
        offsets = torch.from_numpy(workloads.fixed_offsets(N_ELEMENTS, HEADLINE_L).view(np.int32)).cuda()
        graph_ms = time_graph_replay(rs, torch, stream, offsets, copies, best_s, w_best, args.steps, args.warmup)
        print(f"[bench] L={HEADLINE_L} {best} graph replays {graph_ms:.4f} ms per step", file=sys.stderr, flush=True)
    kms = kt_best["mean"]
    # roofline of the dominant kernel: algorithmic bytes over its own mean launch duration
    kgbs = algorithmic_bytes(N_ELEMENTS, HEADLINE_L) / (kms * 1e-3) / 1e9
    probe = probe_copy(rs, torch, stream)
    traffic = measured_traffic(best, w_best)
    # the headline step: graph replays when timed, else the direct launches
    step_ms = graph_ms if graph_ms is not None else ms
    line = {
        "metric": "elements/s and HBM GB/s vs region length (tag vs signal); batched p50/p99 ms",
        "value": N_ELEMENTS / (step_ms * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "boundary-frequency sweep: 2^26 hash-generated u32, fixed region length, "
                               "filter -> expand 0..3 -> per-region u64 sum/min/max/count",
                   "n_elements": N_ELEMENTS, "region_length": HEADLINE_L, "strategy": best,
                   "ensemble_width": w_best, "queue_depth": kt_best["queue_depth"],
                   "input_copies_rotated": COPIES,
                   "timed_launches": ("graph replays of the captured reset + pipeline kernels" if graph_ms is not None
                                      else "direct (reset + pipeline kernel, event pair around each pipeline kernel)")},
        "direct_launches": {
            "ms_per_step": round(ms, 4), "elements_per_s": eps,
            "note": "the same steps launched directly, an event pair around each pipeline kernel (the roofline's "
                    "kernel durations)"},
        "roofline": {"bound": "hbm", "achieved": round(kgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kgbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel_ms": round(kms, 4),
                     "kernel_ms_median": round(kt_best["median"], 4), "kernel_ms_min": round(kt_best["min"], 4),
                     "kernel": f"rs_pipeline<HASH_EXPAND, {best}, ensemble {w_best}>",
                     "algorithmic_bytes_per_launch": algorithmic_bytes(N_ELEMENTS, HEADLINE_L)},
        "hbm_probe": probe,
        "sweep": sweep,
    }
    if partial:
        args.no_variable = args.no_configs = args.no_serving = True
    if not args.headline_only and not args.no_variable:
        line["variable_sweep"] = variable_sweep(rs, torch, stream, copies, args.steps, args.warmup,
                                                parse_widths(args.width).get("tag", 0)
                                                if ":" not in args.width else 0)
    if not args.headline_only and not partial:
        line["output_stream"] = output_stream_rate(rs, torch, stream, copies[0], HEADLINE_L)
        print(f"[bench] output stream: {json.dumps(line['output_stream'])}", file=sys.stderr, flush=True)
    if not args.headline_only and not args.no_configs:
        t_c = time.perf_counter()
        line["configs"] = other_configs(rs, torch, stream)
        print(f"[bench] other configs {time.perf_counter() - t_c:.1f} s: {json.dumps(line['configs'])}",
              file=sys.stderr, flush=True)
    if not args.no_serving and not args.headline_only:
        t_s = time.perf_counter()
        line["serving"] = serving(rs, torch, stream)
        print(f"[bench] serving leg {time.perf_counter() - t_s:.1f} s: {json.dumps(line['serving'])}",
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(HEADLINE_L)
        line["cpu_baseline_threads"] = cpu_baseline_threads(HEADLINE_L)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
