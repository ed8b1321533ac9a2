#!/usr/bin/env python3
"""Benchmark of the gfx950 stable multisplit (one JSON line on stdout).

Default workload: key-value multisplit of n = 2^25 pairs, uint32 keys uniform
over [0, 2^32) (SplitMix64 seed 102), values = original index, m = 32 equal
range buckets f(k) = k >> 27 -- the paper's key-value setting (Section 6:
2^25 uniform 32-bit pairs, delta buckets).  A step is one complete multisplit
call (pre-scan, scan, post-scan) with inputs already resident in HBM.

Reported: Gpairs/s of the whole call; the roofline of the dominant kernel
(the post-scan: 16 algorithmic bytes per pair -- key and value read once and
written once), timed with HIP events on the stream the kernels run on; and
the CPU oracle timed on the host cores.

Other workloads (--workload): keys_2e20_m8, keys_2e28_m<m>, pairs_2e28_m<m>
(m up to 65536; above 256 two stable passes over 8-bit digits of the bucket),
radix_pairs_2e28, radix_keys_2e28, hist_2e<k>_m<m> and histrange_2e<k>_m<m>
(device-wide histograms, even or range bins), and range_2e27_m256: n = 2^27 lognormal
(mu 20, sigma 2) keys saturated to 32 bits (seed 103), 256 range buckets at
quantiles of a 2^16-key sample (seed 1031); sssp_rmat_2e20[_d<delta>]: shortest
paths on an R-MAT graph (Section 7.2); the learned identifier (fit on the
GPU from 2^20 keys, seed 1032) is timed against the binary search over the
same splitters, and `value` is the learned rate.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "multisplit Gkeys/s & Gpairs/s (m=2..256) + % HBM roofline; learned vs binary-search"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pairs_2e25_m32")
    ap.add_argument("--reorder", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--items", type=int, default=0)
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--claim", type=int, default=0, help="batched: work items per queue claim")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cold-reps", type=int, default=10,
                    help="calls timed one by one after writing a 1 GiB scratch buffer (0: skip)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming-copy ceiling measurement")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_ceiling(dev, reps=20, n=1 << 28):
    """Measured streaming-copy rate (GB/s: 4 B read + 4 B written per word)
    of the library's copy kernel on 2^28 words: the practical HBM ceiling the
    roofline fraction is also quoted against."""
    import torch

    from paper_1701_01189_amd import binding as ms
    a = torch.ones(n, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        ms.copy_u32(b, a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ms.copy_u32(b, a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps
    del a, b
    return 8.0 * n / (t * 1e-3) / 1e9


def cold_steps(step, reps, dev):
    """Each call timed alone (HIP events on the call's stream) after a 1 GiB
    scratch buffer is written and then read back, outside the timed region:
    the write evicts the 256 MB Infinity Cache and the L2s, and the read
    evicts the write's own dirty lines, so the timed call neither finds its
    data in a cache nor pays for someone else's write-back.  Returns
    per-call ms."""
    import torch
    scratch = torch.empty(1 << 28, dtype=torch.int32, device=dev)
    hev = HipEvents(2 * reps)
    out = []
    for i in range(reps):
        scratch.fill_(i)
        scratch.sum()
        torch.cuda.synchronize()
        hev.record(2 * i)
        step(None)
        hev.record(2 * i + 1)
        torch.cuda.synchronize()
        out.append(hev.ms(2 * i, 2 * i + 1))
    hev.close()
    del scratch
    return out


def summary(ms_list, units):
    import statistics
    med = statistics.median(ms_list)
    mean = sum(ms_list) / len(ms_list)
    return {"reps": len(ms_list), "median_ms": round(med, 5), "mean_ms": round(mean, 5),
            "value_median": round(units / (med * 1e-3) / 1e9, 3),
            "value_mean": round(units / (mean * 1e-3) / 1e9, 3)}


def workload(name):
    """(kind, n, m, shift, seed): kind in keys, pairs, radix_keys, radix_pairs."""
    if name == "pairs_2e25_m32":
        return "pairs", 1 << 25, 32, 27, 102
    if name == "keys_2e20_m8":
        return "keys", 1 << 20, 8, 29, 101
    if name.startswith("keys_2e28_m") or name.startswith("pairs_2e28_m"):
        m = int(name.split("_m")[1])
        r = (m - 1).bit_length()
        return name.split("_")[0], 1 << 28, m, 32 - r, 100
    if name.startswith("ident_"):
        # ident_keys_2e25_b5: keys uniform in [0, 2^b), identity buckets f(k) = k,
        # m = 2^b (the paper's multisplit-with-identity-buckets sweep, Section 7.1)
        parts = name.split("_")
        bits = int(parts[3][1:])
        return parts[1] + "_ident", 1 << int(parts[2][2:]), 1 << bits, 0, 120 + bits
    if name.startswith("radix_pairs_2e28") or name.startswith("radix_keys_2e28"):
        # radix_pairs_2e28 (8-bit digits) or radix_pairs_2e28_b<bits>; the
        # shift slot carries the digit width
        bits = int(name.split("_b")[1]) if "_b" in name else 8
        return name.split("_2e28")[0], 1 << 28, 1 << bits, bits, 105
    if name == "range_2e27_m256":
        return "range", 1 << 27, 256, 0, 103
    if name == "copy_2e28":
        return "copy", 1 << 28, 1, 0, 7
    if name.startswith("sssp_rmat_2e20"):
        # sssp_rmat_2e20 (delta 800, the fastest measured) or sssp_rmat_2e20_d<delta>
        delta = int(name.split("_d")[1]) if "_d" in name else 800
        return "sssp", 20, 4_800_000, delta, 106
    if name == "batched_4096_m64":
        return "batched", 4096, 64, 8, 104
    if name.startswith("hist_") or name.startswith("histrange_"):
        # hist_2e25_m32: even bins (k >> (32 - log2 m)); histrange_: m-1 random splitters
        size, mm = name.split("_")[1], int(name.split("_m")[1])
        return name.split("_")[0], 1 << int(size[2:]), mm, 32 - (mm - 1).bit_length(), 110
    raise SystemExit("unknown workload %s" % name)


class HipEvents:
    """hipEvent_t handles created through the HIP runtime itself, so that the
    library can record them on the stream its kernels run on."""

    def __init__(self, count):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(count):
            h = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(h.value)

    def record(self, i):
        """Record event i on torch's current stream (the one the library
        launches on)."""
        import torch
        self.hip.hipEventRecord.argtypes = [self.ct.c_void_p, self.ct.c_void_p]
        st = torch.cuda.current_stream().cuda_stream
        if self.hip.hipEventRecord(self.ct.c_void_p(self.ev[i]), self.ct.c_void_p(st)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def ms(self, a, b):
        f = self.ct.c_float()
        rc = self.hip.hipEventElapsedTime(self.ct.byref(f), self.ct.c_void_p(self.ev[a]),
                                          self.ct.c_void_p(self.ev[b]))
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed (%d)" % rc)
        return f.value

    def close(self):
        for h in self.ev:
            self.hip.hipEventDestroy(self.ct.c_void_p(h))


class _Handle:
    def __init__(self, h):
        self.cuda_event = h


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1701_01189_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload_name, n_units):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    counters, or None when none were taken for the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except ValueError:
        return None
    e = t.get("%s/%s" % (kernel, workload_name))
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(kind, keys, vals, m, shift, budget_s):
    import oracle
    n = len(keys)
    reps, t0 = 0, time.perf_counter()
    if kind.startswith("radix"):
        sample = min(n, 1 << 24)
        k, v = keys[:sample], (vals[:sample] if vals is not None else None)
        while True:
            oracle.radix_sort(k, v)
            reps += 1
            el = time.perf_counter() - t0
            if el > budget_s or reps >= 50:
                break
        return {"value": sample * reps / el / 1e9, "unit": "Gpairs/s" if v is not None else
                "Gkeys/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                "sample": "std::stable_sort of the first 2^24 elements, %d reps" % reps}
    mask = m - 1
    if kind == "range":
        sample = min(n, 1 << 24)
        while True:
            oracle.multisplit(keys[:sample], m, oracle.SPLITTERS, splitters=vals)
            reps += 1
            el = time.perf_counter() - t0
            if el > budget_s or reps >= 50:
                break
        return {"value": sample * reps / el / 1e9, "unit": "Gkeys/s", "cores": 1,
                "kind": "oracle", "cpu_model": cpu_model(),
                "sample": "the first 2^24 keys, std::upper_bound buckets, %d reps" % reps}
    while True:
        oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals, shift=shift, mask=mask)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 50:
            break
    return {"value": n * reps / el / 1e9, "unit": "Gpairs/s" if vals is not None else "Gkeys/s",
            "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "the full %d-element input, %d reps, single-threaded" % (n, reps)}


def time_steps(step, K, warmup):
    """Warm-up, then K timed calls; per call a list of 4 stage events."""
    import torch
    for _ in range(warmup):
        step(None)
    hev = HipEvents(4 * K)
    evs = [[_Handle(hev.ev[4 * i + j]) for j in range(4)] for i in range(K)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(K):
        step(evs[i])
    t1.record(stream)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1) / K
    stage = [sum(hev.ms(4 * i + s, 4 * i + s + 1) for i in range(K)) / K for s in range(3)]
    hev.close()
    return total, stage


def bench_batched(args, num, m, shift, seed, dev):
    """4096 independent key-value instances, sizes log-uniform in [2^8, 2^20]
    (seed 104), keys uniform (seed 104000 + i), values = index within the
    instance, m = 64, f(k) = (k >> 8) & 63; the tuning comes from the
    autotuner; the call is captured in a HIP graph and the replays are timed."""
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs, tuning
    sizes = inputs.batched_sizes(seed, num)
    seg = inputs.segment_offsets(sizes)
    keys, vals = inputs.batched_pairs(seed, sizes)
    total = len(keys)
    dk = torch.from_numpy(keys.view(np.int32)).to(dev)
    dv = torch.from_numpy(vals.view(np.int32)).to(dev)
    ds = torch.from_numpy(seg.astype(np.int64)).to(dev)
    fn = ms.BucketFn.shift_mask(shift, m - 1)
    if args.reorder or args.waves or args.items or args.claim:
        opt = ms.Options(waves_per_block=args.waves, items_per_lane=args.items,
                         batch_claim=args.claim)
        tune = {"source": "command line"}
    else:
        opt, tune = tuning.tuned_options(ms.OP_BATCHED, dk, dv, m, fn=fn, seg=ds)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    off = torch.empty(num * (m + 1), dtype=torch.int32, device=dev)
    need = ms.workspace_size(ms.OP_BATCHED, total, m, num, opt)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ms.batched(dk, dv, ds, m, fn, keys_out=ko, vals_out=vo, offsets=off, options=opt, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ms.batched(dk, dv, ds, m, fn, keys_out=ko, vals_out=vo, offsets=off, options=opt, ws=ws)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        g.replay()
    t1.record()
    torch.cuda.synchronize()
    t = t0.elapsed_time(t1) / args.steps
    status = ms.batched_status(ws)
    value = total / (t * 1e-3) / 1e9
    gbps = 20.0 * total / (t * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "instances": num, "total_pairs": total, "m": m,
                   "bucket": "(k >> 8) & 63", "seed": seed, "hipgraph": True,
                   "tuning": {"waves_per_block": opt.waves_per_block,
                              "items_per_lane": opt.items_per_lane,
                              "batch_claim": opt.batch_claim}, "tuner": tune},
        "status": status,
        "roofline": {"bound": "hbm", "kernel": "batched_kernel (pre-scan and post-scan)",
                     "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for("batched", args.workload, total),
                     "bytes_per_unit": 20},
    }
    print(json.dumps(line), flush=True)


def bench_hist(args, kind, n, m, shift, seed, dev):
    """Device-wide histogram (Section 7.3) of n uniform 32-bit keys: even bins
    f(k) = k >> (32 - log2 m), or range bins over m-1 sorted random splitters
    (seed 113), as in the paper's Even and Range experiments (2^25 elements,
    m <= 256).  One step = one ms_histogram call (zero the output, pre-scan with
    atomic accumulation)."""
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    keys = inputs.uniform_u32(seed, n)
    dk = torch.from_numpy(keys.view(np.int32)).to(dev)
    spl = np.sort(inputs.uniform_u32(113, m - 1)) if kind == "histrange" else None
    ds = torch.from_numpy(spl.view(np.int32)).to(dev) if spl is not None else None
    fn = ms.BucketFn.splitter(ds) if ds is not None else ms.BucketFn.shift_mask(shift, m - 1)
    base = dict(reorder=args.reorder, waves_per_block=args.waves, items_per_lane=args.items,
                max_chunks=args.chunks)
    hist = torch.empty(m, dtype=torch.int32, device=dev)
    ws = torch.empty(max(256, ms.workspace_size(ms.OP_HISTOGRAM, n, m, 0, ms.Options(**base))),
                     dtype=torch.uint8, device=dev)

    def step(ev):
        ms.histogram(dk, m, fn, hist=hist, options=ms.Options(stage_events=ev, **base), ws=ws)
    t_eager, st = time_steps(step, args.steps, args.warmup)
    # A call is ~20-200 us of GPU work, close to the host's own cost of a
    # call from Python; replaying the call from a HIP graph measures the GPU.
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(None)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(None)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / args.steps
    value = n / (t * 1e-3) / 1e9
    pre_gbps = 4.0 * n / (st[0] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m,
                   "bins": "range (m-1 random splitters)" if spl is not None else "even (k >> %d)" % shift,
                   "seed": seed, **base},
        "hipgraph": True,
        "eager_value": round(n / (t_eager * 1e-3) / 1e9, 3),
        "stage_ms": {"prescan": round(st[0], 5), "reduce": round(st[1], 5)},
        "roofline": {"bound": "hbm", "kernel": "prescan", "achieved": round(pre_gbps, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(pre_gbps / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for("prescan", args.workload, n), "bytes_per_unit": 4},
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = min(n, 1 << 24)
        reps, t0 = 0, time.perf_counter()
        while True:
            if spl is not None:
                oracle.histogram(keys[:sample], m, oracle.SPLITTERS, splitters=spl)
            else:
                oracle.histogram(keys[:sample], m, oracle.SHIFT_MASK, shift=shift, mask=m - 1)
            reps += 1
            el = time.perf_counter() - t0
            if el > args.cpu_seconds or reps >= 50:
                break
        line["cpu_baseline"] = {"value": sample * reps / el / 1e9, "unit": "Gkeys/s", "cores": 1,
                                "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": "the first 2^24 keys, %d reps" % reps}
    print(json.dumps(line), flush=True)


def bench_sssp(args, scale, n_edges, delta, seed, dev):
    """Delta-stepping shortest paths with multisplit bucketing (Section 7.2)
    on the R-MAT graph of the paper's evaluation: 2^scale vertices, n_edges
    undirected edges drawn with (a, b, c, d) = (0.5, 0.1, 0.1, 0.3), each
    stored in both directions, integer weights uniform in [0, 1000], source
    vertex 0, 10 buckets.  One step = one complete ms_sssp call.  The rate is
    the paper's MTEPS: stored (directed) edges over the call's time."""
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    row, col, wt = inputs.rmat_graph(seed, scale, n_edges)
    ne = len(col)
    r = torch.from_numpy(row.astype(np.int64)).to(dev)
    c = torch.from_numpy(col.view(np.int32)).to(dev)
    w = torch.from_numpy(wt.view(np.int32)).to(dev)
    dist = torch.empty(len(row) - 1, dtype=torch.int32, device=dev)
    ws = torch.empty(ms.sssp_workspace_size(len(row) - 1, ne, 10), dtype=torch.uint8, device=dev)
    stats = {}

    def step(ev):
        if ev is not None:
            ev.record(0)
        _, st = ms.sssp(r, c, w, 0, delta=delta, num_buckets=10, dist=dist, ws=ws)
        if ev is not None:
            ev.record(1)
        stats.update(st)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    ev = HipEvents(2)
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(ev)
        torch.cuda.synchronize()
        times.append(ev.ms(0, 1))
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    ev.close()
    t = sum(times) / len(times)
    # Algorithmic bytes of a run: each pending entry is multisplit as a pair
    # (20 B: key read by the pre-scan, pair read and written by the
    # post-scan) and filtered (12 B: pair and its vertex's distance); each
    # relaxed edge reads its target and weight and updates a distance (16 B);
    # each improvement appends a pair (8 B).
    byts = 32 * stats["items_split"] + 16 * stats["edges_relaxed"] + 8 * stats["pushes"]
    gbps = byts / (t * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(ne / (t * 1e-3) / 1e6, 1), "unit": "MTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": "rmat", "scale": scale,
                   "vertices": len(row) - 1, "edges_stored": ne, "delta": delta, "buckets": 10,
                   "source": 0, "seed": seed},
        "wall_ms_per_step": round(wall, 4),
        "sssp": stats,
        "roofline": {"bound": "hbm", "kernel": "whole call", "achieved": round(gbps, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "traffic": None, "bytes_per_run": byts},
    }
    if not args.no_cpu_baseline:
        import oracle
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.sssp(row, col, wt, 0)
            reps += 1
            el = time.perf_counter() - t0
            if el > args.cpu_seconds or reps >= 20:
                break
        line["cpu_baseline"] = {"value": round(ne * reps / el / 1e6, 2), "unit": "MTEPS",
                                "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": "the full graph, %d Dijkstra runs" % reps}
    print(json.dumps(line), flush=True)


def bench_copy(args, n, dev):
    """Streaming copy of n words (the measured HBM ceiling, and the known
    byte count that scales the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch

    from paper_1701_01189_amd import binding as ms
    a = torch.ones(n, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ms.copy_u32(b, a)
    hev = HipEvents(2)
    hip = hev.hip
    import ctypes
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    torch.cuda.synchronize()
    hip.hipEventRecord(ctypes.c_void_p(hev.ev[0]), ctypes.c_void_p(stream.cuda_stream))
    for _ in range(args.steps):
        ms.copy_u32(b, a)
    hip.hipEventRecord(ctypes.c_void_p(hev.ev[1]), ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    t = hev.ms(0, 1) / args.steps
    hev.close()
    gbps = 8.0 * n / (t * 1e-3) / 1e9
    print(json.dumps({"metric": "streaming copy GB/s (ceiling probe)", "value": round(gbps, 1),
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(t, 5), "higher_is_better": True, "dtype": "u32",
                      "data": "synthetic", "config": {"workload": "copy_2e28", "n": n,
                                                      "bytes_per_launch": 8 * n}}), flush=True)


def bench_range(args, n, m, seed, dev):
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    keys = inputs.lognormal_u32(seed, n)
    spl = inputs.quantile_splitters(inputs.lognormal_u32(1031, 1 << 16), m)
    fit = inputs.lognormal_u32(1032, 1 << 20)
    dk = torch.from_numpy(keys.view(np.int32)).to(dev)
    ds = torch.from_numpy(spl.view(np.int32)).to(dev)
    dfit = torch.from_numpy(fit.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    model = ms.learned_fit(dfit, ds, m)
    torch.cuda.synchronize()
    fit_ms = (time.perf_counter() - f0) * 1e3
    ok = torch.empty_like(dk)
    off = torch.empty(m + 1, dtype=torch.int32, device=dev)
    base = dict(reorder=args.reorder, waves_per_block=args.waves, items_per_lane=args.items,
                max_chunks=args.chunks)
    ws = torch.empty(max(256, ms.workspace_size(ms.OP_KEYS, n, m, 0, ms.Options(**base))),
                     dtype=torch.uint8, device=dev)
    res = {}
    for name, fn in (("learned", ms.BucketFn.learned(ds, model)),
                     ("binary_search", ms.BucketFn.splitter(ds))):
        def step(ev, fn=fn):
            ms.keys(dk, m, fn, keys_out=ok, offsets=off, options=ms.Options(stage_events=ev, **base),
                    ws=ws)
        res[name] = time_steps(step, args.steps, args.warmup)
    miss = torch.zeros(1, dtype=torch.int64, device=dev)
    ms.keys(dk, m, ms.BucketFn.learned(ds, model), keys_out=ok, offsets=off,
            options=ms.Options(mispredicts=miss, **base), ws=ws)
    torch.cuda.synchronize()
    lt, lst = res["learned"]
    bt, bst = res["binary_search"]
    value = n / (lt * 1e-3) / 1e9
    post_gbps = n * 8 / (lst[2] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(lt, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "bucket": "learned range",
                   "keys": "lognormal(20,2) saturated", "seed": seed, **base},
        "stage_ms": {"prescan": round(lst[0], 5), "scan": round(lst[1], 5),
                     "postscan": round(lst[2], 5)},
        "binary_search": {"value": round(n / (bt * 1e-3) / 1e9, 3), "ms_per_step": round(bt, 5),
                          "stage_ms": {"prescan": round(bst[0], 5), "scan": round(bst[1], 5),
                                       "postscan": round(bst[2], 5)}},
        "learned_speedup": round(bt / lt, 4),
        "mispredict_rate": round(int(miss.item()) / n, 5),
        "fit_ms_wall": round(fit_ms, 3),
        "roofline": {"bound": "hbm", "kernel": "postscan", "achieved": round(post_gbps, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(post_gbps / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for("postscan", args.workload, n), "bytes_per_unit": 8},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline("range", keys, spl, m, 0, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the multisplit library runs on one GPU; only --gpus 1 is "
              "measured (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import build as b
    from paper_1701_01189_amd import inputs

    if not os.path.exists(b.LIB):
        b.build(force=True)
    kind, n, m, shift, seed = workload(args.workload)
    kv = kind.startswith("pairs") or kind == "radix_pairs"
    dev = torch.device("cuda:0")
    if kind == "range":
        return bench_range(args, n, m, seed, dev)
    if kind == "copy":
        return bench_copy(args, n, dev)
    if kind == "batched":
        return bench_batched(args, n, m, shift, seed, dev)
    if kind == "sssp":
        return bench_sssp(args, n, m, shift, seed, dev)
    if kind in ("hist", "histrange"):
        return bench_hist(args, kind, n, m, shift, seed, dev)
    ident = kind.endswith("_ident")
    if ident:
        kind = kind[:-len("_ident")]
    keys = inputs.uniform_u32(seed, n)
    if ident:
        keys &= np.uint32(m - 1)
    vals = inputs.index_values(n) if kv else None
    dk = torch.from_numpy(keys.view(np.int32)).to(dev)
    dv = torch.from_numpy(vals.view(np.int32)).to(dev) if kv else None
    ok = torch.empty_like(dk)
    ov = torch.empty_like(dv) if kv else None
    off = torch.empty(m + 1, dtype=torch.int32, device=dev)
    opt = ms.Options(reorder=args.reorder, waves_per_block=args.waves,
                     items_per_lane=args.items, max_chunks=args.chunks)
    radix = kind.startswith("radix")
    op = (ms.OP_RADIX_SORT_PAIRS if kv else ms.OP_RADIX_SORT) if radix else \
        (ms.OP_PAIRS if kv else ms.OP_KEYS)
    ws = torch.empty(max(256, ms.workspace_size(op, n, m, 0, opt)), dtype=torch.uint8,
                     device=dev)
    # powers of two: shift/mask; other m: delta buckets floor(k / ceil(2^32 / m))
    pow2 = m & (m - 1) == 0
    fn = ms.BucketFn.shift_mask(shift, m - 1) if pow2 else ms.BucketFn.div(-(-(1 << 32) // m))

    def step(o):
        if radix:
            ms.radix_sort(dk, dv, shift, keys_out=ok, vals_out=ov, options=o, ws=ws)
        elif kv:
            ms.pairs(dk, dv, m, fn, keys_out=ok, vals_out=ov, offsets=off, options=o, ws=ws)
        else:
            ms.keys(dk, m, fn, keys_out=ok, offsets=off, options=o, ws=ws)

    for _ in range(args.warmup):
        step(opt)
    K = args.steps
    hev = HipEvents(4 * K)
    evs = [[_Handle(hev.ev[4 * i + j]) for j in range(4)] for i in range(K)]
    cev = HipEvents(K + 1)  # call boundaries (a radix sort records stages of its last pass only)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t_start.record(stream)
    for i in range(K):
        o = ms.Options(reorder=args.reorder, waves_per_block=args.waves,
                       items_per_lane=args.items, max_chunks=args.chunks, stage_events=evs[i])
        cev.record(i)
        step(o)
    cev.record(K)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / K
    stage = [0.0, 0.0, 0.0]
    for i in range(K):
        for s in range(3):
            stage[s] += hev.ms(4 * i + s, 4 * i + s + 1) / K
    per_call = [cev.ms(i, i + 1) for i in range(K)]
    hev.close()
    cev.close()
    cold = None
    if args.cold_reps > 0:
        cold = summary(cold_steps(lambda _ev: step(opt), args.cold_reps, dev), n)
    # The same call captured in a HIP graph and replayed K times: the GPU's
    # own time per call, without the host's cost of issuing it from Python.
    # For small inputs (2^20 keys: ~25 us of GPU work) the eager loop measures
    # the host, so `value` is taken from the replays there.
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(opt)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(opt)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(K):
        graph.replay()
    g1.record()
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / K
    del graph
    ceiling = None if args.no_ceiling else copy_ceiling(dev)
    # correctness spot check of the last step against the properties of the
    # unique stable result is done by the tests; here only a cheap sanity check
    units = n
    small = n <= (1 << 22)
    timed_ms = graph_ms if small else ms_per_step
    value = units / (timed_ms * 1e-3) / 1e9
    # dominant kernel: the post-scan (of the last pass for the radix sort)
    post_bytes = n * (16 if kv else 8)
    post_ms = stage[2]
    achieved = post_bytes / (post_ms * 1e-3) / 1e9
    traffic = traffic_for("postscan", args.workload, n)
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpairs/s" if kv else "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(timed_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "timing": "hipgraph replays" if small else "eager calls",
        "eager_value": round(units / (ms_per_step * 1e-3) / 1e9, 3),
        "graph_value": round(units / (graph_ms * 1e-3) / 1e9, 3),
        "config": {"workload": args.workload, "n": n, "m": m,
                   "bucket": ("radix %d x %d-bit digits" % (-(-32 // shift), shift) if radix else
                              "identity (keys < m)" if ident else
                              "shift_mask" if pow2 else "delta ceil(2^32/m)"),
                   "shift": shift, "kv": kv, "seed": seed,
                   "reorder": args.reorder, "waves_per_block": args.waves,
                   "items_per_lane": args.items},
        "stage_ms": {"prescan": round(stage[0], 5), "scan": round(stage[1], 5),
                     "postscan": round(stage[2], 5)},
        "wall_s": round(wall, 4),
        "roofline": {"bound": "hbm", "kernel": "postscan", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "bytes_per_unit": 16 if kv else 8,
                     "whole_call_algorithmic_GBps": round(n * (20 if kv else 12) /
                                                          (timed_ms * 1e-3) / 1e9, 1)},
        "warm_per_call": summary(per_call, n),
    }
    if cold is not None:
        line["cold_per_call"] = cold
    if ceiling is not None:
        line["roofline"]["copy_ceiling_GBps"] = round(ceiling, 1)
        line["roofline"]["frac_of_copy_ceiling"] = round(achieved / ceiling, 4)
    if radix:
        line["roofline"]["whole_call_algorithmic_GBps"] = round(
            n * -(-32 // shift) * (20 if kv else 12) / (timed_ms * 1e-3) / 1e9, 1)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(kind, keys, vals, m, shift, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
