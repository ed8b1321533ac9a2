#!/usr/bin/env python3
"""Benchmark of the gfx950 stable multisplit (one JSON line on stdout).

Default workload (`headline`): key-only stable multisplit of n = 2^28 uint32
keys uniform over [0, 2^32) (SplitMix64 seed 100) into m = 32 delta buckets
f(k) = k >> 27, calls issued back to back with the keys already in HBM.  A
step is one complete call (pre-scan, scan of H, post-scan).  `value` is
Gkeys/s over K back-to-back calls timed between two events with nothing else
on the stream; the per-stage times come from a second pass of K calls that
record stage events.

The same line carries, under `rows`, every other measured configuration, each
with its own roofline and CPU-oracle baseline:
  * sweep: key-only and key-value, n = 2^28, m = 2, 4, ..., 256;
  * skew: m = 256 with binomial B(255, 1/2) and 1/4-uniform bucket
    distributions next to uniform buckets, n = 2^25 (Section 6.4);
  * keys_2e20_m8: n = 2^20, m = 8 (HIP-graph replays: a call is ~20 us);
  * pairs_2e25_m32: the block- / wave- / no-reorder sweep over tile shapes
    (Section 6.2, WMS against BMS);
  * range_2e27_m256: 2^27 lognormal keys, 256 range buckets, learned bucket
    identifier against binary search over the splitters;
  * batched_4096_m64: 4096 key-value instances in one persistent launch,
    autotuned, HIP-graph replays;
  * radix_pairs_2e28: LSD radix sort of 2^28 pairs, 4 passes of 8 bits.

Byte model (Section 6.2.2, speed of light): a key-only multisplit must move
12 bytes per key (read by the pre-scan, read by the post-scan, written), a
key-value one 20 bytes per pair.  `roofline` is that of the dominant kernel,
the post-scan (8 bytes per key, 16 per pair); `whole_call` puts the call's
12 or 20 bytes per element against the same 8 TB/s peak.

Single workloads (--workload NAME) print one line each: keys_2e28_m<m>,
pairs_2e28_m<m> (m up to 65536), keys_2e20_m8, pairs_2e25_m32,
skew_{binomial,alpha,uniform}_{keys,pairs}_2e25_m256, ident_{keys,pairs}_2e25_b<b>,
radix_{pairs,keys}_2e28[_b<bits>], range_2e27_m256, batched_4096_m64,
hist_2e<k>_m<m>, histrange_2e<k>_m<m>, sssp_rmat_2e20[_d<delta>], copy_2e28.
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

# Section 6.2.2: three 4-byte global accesses per key, five per key-value pair.
BYTES_PER_KEY = 12
BYTES_PER_PAIR = 20
# The post-scan's share: read the key (and value) again, write it.
POST_BYTES_PER_KEY = 8
POST_BYTES_PER_PAIR = 16
GATE_FRAC = 0.60  # key-only, m <= 32: at least 60 % of the HBM peak, whole call
GRAPH_CALLS = 10  # calls captured per HIP graph when replays are timed


def progress(msg):
    """A line on stderr after each measured row (the JSON line is stdout's)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def call_bytes(kv):
    return BYTES_PER_PAIR if kv else BYTES_PER_KEY


def sol_rate(bandwidth_gbps, kv):
    """Speed-of-light rate (G elements/s) at a bandwidth, by the byte model."""
    return bandwidth_gbps / call_bytes(kv)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--reorder", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--items", type=int, default=0)
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--claim", type=int, default=0, help="batched: work items per queue claim")
    ap.add_argument("--keep-ids", type=int, default=1,
                    help="range buckets: the pre-scan keeps bucket ids for the post-scan")
    ap.add_argument("--device-warmup-ms", type=float, default=200.0,
                    help="streaming copies on scratch buffers right before each row's "
                         "warm-up calls, so that the GPU's clocks have settled (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle time budget of the headline (or single workload)")
    ap.add_argument("--row-cpu-seconds", type=float, default=1.0,
                    help="oracle time budget of each sub-row")
    ap.add_argument("--cold-reps", type=int, default=0,
                    help="single workloads: calls timed one by one after a 1 GiB scratch "
                         "write and read-back (informational; 0: skip)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming-copy ceiling measurement")
    ap.add_argument("--rows", default="sweep,skew,config1,config2,config3,config4,config5",
                    help="headline: comma-separated sub-row groups to measure")
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


def device_warmup(ms_budget, n=1 << 27):
    """Keeps the GPU busy with the library's streaming copy (two scratch
    buffers of its own, 512 MiB each) for about ms_budget milliseconds right
    before a row's warm-up calls.  After host-side work (input generation, the
    CPU baseline) the GPU has been idle, and the first calls that follow run
    slower until its clocks settle (2^28 keys, m = 32: 0.754 ms per call
    against 0.707 ms in later passes).  Nothing the timed calls read or write
    is touched or cached by it."""
    import time

    import torch

    from paper_1701_01189_amd import binding as ms
    if ms_budget <= 0:
        return 0.0
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms_budget:
        for _ in range(20):
            ms.copy_u32(b, a)
        torch.cuda.synchronize()
    del a, b
    return (time.perf_counter() - t0) * 1e3


def cold_steps(step, reps, dev):
    """Each call timed alone after a 1 GiB scratch buffer is written and read
    back outside the timed region (caches hold none of the call's data).  The
    timed region ends when the call's last kernel ends, which can be before
    all of its dirty lines have reached HBM: informational only, never the
    reported value."""
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
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
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


def traffic_for(kernel, workload_name):
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


def roofline(kernel, workload_name, algo_bytes, kernel_ms, ceiling=None):
    achieved = algo_bytes / (kernel_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
         "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
         "traffic": traffic_for(kernel, workload_name),
         "algorithmic_bytes_per_launch": int(algo_bytes),
         "avg_launch_ms": round(kernel_ms, 5)}
    if ceiling:
        r["copy_ceiling_GBps"] = round(ceiling, 1)
        r["frac_of_copy_ceiling"] = round(achieved / ceiling, 4)
    return r


def whole_call(n, kv, call_ms, passes=1):
    b = n * passes * call_bytes(kv)
    gbps = b / (call_ms * 1e-3) / 1e9
    return {"bytes_per_unit": passes * call_bytes(kv), "achieved": round(gbps, 1),
            "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4)}


def _oracle_rate(run, units, budget_s, max_reps=50):
    reps, t0 = 0, time.perf_counter()
    while True:
        run()
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= max_reps:
            break
    return units * reps / el / 1e9, reps


def cpu_baseline(kind, keys, vals, m, shift, budget_s, sample_max=None, splitters=None):
    """The CPU oracle (single-threaded) on a bounded sample of the same input."""
    import oracle
    n = len(keys)
    sample = n if sample_max is None else min(n, sample_max)
    k = keys[:sample]
    v = vals[:sample] if vals is not None else None
    unit = "Gpairs/s" if v is not None else "Gkeys/s"
    if kind.startswith("radix"):
        rate, reps = _oracle_rate(lambda: oracle.radix_sort(k, v), sample, budget_s)
        what = "std::stable_sort of the first %d elements, %d reps" % (sample, reps)
    elif splitters is not None:
        rate, reps = _oracle_rate(
            lambda: oracle.multisplit(k, m, oracle.SPLITTERS, vals=v, splitters=splitters),
            sample, budget_s)
        what = "the first %d keys, upper-bound buckets, %d reps" % (sample, reps)
    else:
        rate, reps = _oracle_rate(
            lambda: oracle.multisplit(k, m, oracle.SHIFT_MASK, vals=v, shift=shift, mask=m - 1),
            sample, budget_s)
        what = "the first %d elements, %d reps" % (sample, reps)
    return {"value": round(rate, 5), "unit": unit, "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "sample": what + ", single-threaded"}


DEVICE_WARMUP_MS = 0.0


def time_calls(step, K, warmup, stages=True, graph=False):
    """Warm-up, then K back-to-back calls between two events (nothing else on
    the stream).  With stages, a second pass of K calls records the four
    stage events of each call (the radix sort records its last pass only) and
    the mean stage times are returned.  With graph, the call is also captured
    in a HIP graph and K replays are timed."""
    import torch
    stream = torch.cuda.current_stream()
    device_warmup(DEVICE_WARMUP_MS)
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(K):
        step(None)
    t1.record(stream)
    torch.cuda.synchronize()
    out = {"ms": t0.elapsed_time(t1) / K}
    if stages:
        hev = HipEvents(4 * K)
        evs = [[_Handle(hev.ev[4 * i + j]) for j in range(4)] for i in range(K)]
        torch.cuda.synchronize()
        t0.record(stream)
        for i in range(K):
            step(evs[i])
        t1.record(stream)
        torch.cuda.synchronize()
        out["stage"] = [sum(hev.ms(4 * i + s, 4 * i + s + 1) for i in range(K)) / K
                        for s in range(3)]
        # per call in the second pass (the one that records the stage events):
        # the first timed calls after the warm-up run slower than later ones
        out["stage_pass_ms"] = t0.elapsed_time(t1) / K
        hev.close()
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step(None)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        # GRAPH_CALLS calls per graph: a captured loop of calls, as a serving
        # loop would replay it (one call per graph measures the runtime's
        # cost of launching a graph, tens of microseconds, instead)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(GRAPH_CALLS):
                step(None)
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        reps = max(1, K // GRAPH_CALLS)
        t0.record(stream)
        for _ in range(reps):
            g.replay()
        t1.record(stream)
        torch.cuda.synchronize()
        out["graph_ms"] = t0.elapsed_time(t1) / (reps * GRAPH_CALLS)
        del g
    return out


# ---------------------------------------------------------------------------
# multisplit rows
# ---------------------------------------------------------------------------
def multisplit_row(args, name, dk, dv, m, fn, shape=(0, 0, 0), graph=False, cpu=None,
                   ceiling=None, radix_bits=0, tune=False, keep_ids=0):
    """One multisplit (or radix sort when radix_bits) workload on resident
    device inputs.  With tune, the shape comes from the autotuner through
    its cache.  Returns the row dict."""
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import tuning
    n = dk.numel()
    kv = dv is not None
    ok = torch.empty_like(dk)
    ov = torch.empty_like(dv) if kv else None
    mm = (1 << radix_bits) if radix_bits else m
    off = torch.empty(mm + 1, dtype=torch.int32, device=dk.device)
    op = ((ms.OP_RADIX_SORT_PAIRS if kv else ms.OP_RADIX_SORT) if radix_bits else
          (ms.OP_PAIRS if kv else ms.OP_KEYS))
    tuned = None
    if tune and shape == (0, 0, 0):
        topt, tuned = tuning.tuned_options(op, dk, dv, radix_bits if radix_bits else m, fn=fn,
                                           keep_bucket_ids=keep_ids)
        shape = (topt.reorder, topt.waves_per_block, topt.items_per_lane)
    base = dict(reorder=shape[0], waves_per_block=shape[1], items_per_lane=shape[2],
                max_chunks=args.chunks, keep_bucket_ids=keep_ids)
    ws = torch.empty(max(256, ms.workspace_size(op, n, mm, 0, ms.Options(**base))),
                     dtype=torch.uint8, device=dk.device)
    opt_plain = ms.Options(**base)

    def step(ev):
        o = opt_plain if ev is None else ms.Options(stage_events=ev, **base)
        if radix_bits:
            ms.radix_sort(dk, dv, radix_bits, keys_out=ok, vals_out=ov, options=o, ws=ws)
        elif kv:
            ms.pairs(dk, dv, m, fn, keys_out=ok, vals_out=ov, offsets=off, options=o, ws=ws)
        else:
            ms.keys(dk, m, fn, keys_out=ok, offsets=off, options=o, ws=ws)

    t = time_calls(step, args.steps, args.warmup, stages=True, graph=graph)
    call_ms = t["graph_ms"] if graph else t["ms"]
    passes = -(-32 // radix_bits) if radix_bits else 1
    value = n / (call_ms * 1e-3) / 1e9
    post_ms = t["stage"][2]
    kern = "postscan"
    row = {
        "workload": name, "n": n, "m": mm, "kv": kv,
        "value": round(value, 3), "unit": "Gpairs/s" if kv else "Gkeys/s",
        "ms_per_call": round(call_ms, 5),
        "timing": ("hipgraph replays, %d calls per graph" % GRAPH_CALLS) if graph else
                  "back-to-back eager calls",
        "stage_ms": {"prescan": round(t["stage"][0], 5), "scan": round(t["stage"][1], 5),
                     "postscan": round(post_ms, 5)},
        "roofline": roofline(kern, name, n * (POST_BYTES_PER_PAIR if kv else POST_BYTES_PER_KEY),
                             post_ms, ceiling),
        "whole_call": whole_call(n, kv, call_ms, passes),
    }
    if "stage_pass_ms" in t:
        row["second_pass_ms_per_call"] = round(t["stage_pass_ms"], 5)
    if radix_bits:
        row["passes"] = passes
        row["stage_ms_note"] = "stages of the last pass"
    if graph:
        row["eager_ms_per_call"] = round(t["ms"], 5)
    if shape != (0, 0, 0):
        row["shape"] = {"reorder": ["auto", "block", "wave", "none"][shape[0]],
                        "waves_per_block": shape[1], "windows_per_wave": shape[2]}
    if keep_ids:
        row["kept_bucket_ids"] = True
        row["bytes_per_unit"] = call_bytes(kv) + 2  # + 1 B id written, 1 B read
    if tuned is not None:
        row["tuner"] = tuned
    if cpu is not None and not args.no_cpu_baseline:
        row["cpu_baseline"] = cpu()
    del ok, ov, ws
    progress("%s: %.3f %s" % (name, row["value"], row["unit"]))
    return row


def keys_device(keys, vals, dev):
    import numpy as np
    import torch
    dk = torch.from_numpy(keys.view(np.int32)).to(dev)
    dv = torch.from_numpy(vals.view(np.int32)).to(dev) if vals is not None else None
    return dk, dv


def pow2_fn(m):
    from paper_1701_01189_amd import binding as ms
    r = (m - 1).bit_length()
    if m & (m - 1) == 0:
        return ms.BucketFn.shift_mask(32 - r if r else 0, m - 1), 32 - r
    return ms.BucketFn.div(-(-(1 << 32) // m)), None


def rows_sweep(args, keys, dev, ceiling, sizes=(2, 4, 8, 16, 32, 64, 128, 256), headline=None):
    """Key-only and key-value at n = 2^28, m = 2..256, shift buckets."""
    from paper_1701_01189_amd import inputs
    out = {}
    dk, _ = keys_device(keys, None, dev)
    for m in sizes:
        name = "keys_2e28_m%d" % m
        if headline is not None and name == headline["workload"]:
            out[name] = {k: v for k, v in headline.items() if k != "rows"}
            continue
        fn, shift = pow2_fn(m)
        out[name] = multisplit_row(
            args, name, dk, None, m, fn, ceiling=ceiling,
            cpu=lambda m=m, shift=shift: cpu_baseline("keys", keys, None, m, shift,
                                                      args.row_cpu_seconds, 1 << 22))
    vals = inputs.index_values(len(keys))
    _, dv = keys_device(keys, vals, dev)
    for m in sizes:
        name = "pairs_2e28_m%d" % m
        fn, shift = pow2_fn(m)
        out[name] = multisplit_row(
            args, name, dk, dv, m, fn, ceiling=ceiling,
            cpu=lambda m=m, shift=shift: cpu_baseline("pairs", keys, vals, m, shift,
                                                      args.row_cpu_seconds, 1 << 22))
    del dk, dv
    return out


def rows_skew(args, dev, ceiling):
    """m = 256 with skewed bucket distributions (Section 6.4, Table of
    distributions): binomial B(255, 1/2) and 1/4-uniform, beside uniform
    buckets, n = 2^25 as in the paper, keys and pairs."""
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    n, m = 1 << 25, 256
    out = {}
    vals = inputs.index_values(n)
    fn = ms.BucketFn.shift_mask(24, 255)
    for dist in ("binomial", "alpha", "uniform"):
        keys = inputs.skewed_bucket_keys(100, n, m, dist)
        dk, dv = keys_device(keys, vals, dev)
        for kv in (False, True):
            name = "skew_%s_%s_2e25_m256" % (dist, "pairs" if kv else "keys")
            out[name] = multisplit_row(
                args, name, dk, dv if kv else None, m, fn, ceiling=ceiling,
                cpu=lambda keys=keys, kv=kv: cpu_baseline(
                    "pairs" if kv else "keys", keys, vals if kv else None, m, 24,
                    args.row_cpu_seconds, 1 << 22))
            out[name]["distribution"] = {"binomial": "bucket ~ B(255, 1/2)",
                                         "alpha": "1/4 uniform, else one bucket",
                                         "uniform": "uniform"}[dist]
        del dk, dv
    return out


def row_config1(args, dev, ceiling):
    """n = 2^20 keys (seed 101), m = 8, f = k >> 29: a call is a few tens of
    microseconds, so HIP-graph replays time the GPU rather than the host."""
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    keys = inputs.uniform_u32(101, 1 << 20)
    dk, _ = keys_device(keys, None, dev)
    row = multisplit_row(args, "keys_2e20_m8", dk, None, 8, ms.BucketFn.shift_mask(29, 7),
                         graph=True, ceiling=ceiling, tune=True,
                         cpu=lambda: cpu_baseline("keys", keys, None, 8, 29,
                                                  args.row_cpu_seconds))
    row["note"] = "latency bound: 12.6 MB fits in the 256 MB memory-side cache"
    return row


CONFIG2_SHAPES = [(0, 0, 0), (1, 4, 16), (1, 8, 8), (1, 8, 4), (1, 4, 8), (1, 16, 8),
                  (2, 8, 8), (2, 4, 16), (3, 8, 8)]


def rows_config2(args, dev, ceiling):
    """n = 2^25 pairs (seed 102), values = index, m = 32, f = k >> 27; block-,
    wave- and no-reorder over tile shapes."""
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    n = 1 << 25
    keys = inputs.uniform_u32(102, n)
    vals = inputs.index_values(n)
    dk, dv = keys_device(keys, vals, dev)
    fn = ms.BucketFn.shift_mask(27, 31)
    out = {}
    cpu_once = {}

    def cpu():
        if "v" not in cpu_once:
            cpu_once["v"] = cpu_baseline("pairs", keys, vals, 32, 27, args.row_cpu_seconds)
        return cpu_once["v"]
    for shape in CONFIG2_SHAPES:
        tag = "auto" if shape == (0, 0, 0) else "%s_%dx%d" % (
            ["", "block", "wave", "none"][shape[0]], shape[1], shape[2])
        name = "pairs_2e25_m32"
        r = multisplit_row(args, name, dk, dv, 32, fn, shape=shape, ceiling=ceiling, cpu=cpu)
        out["pairs_2e25_m32_" + tag] = r
    return out


def row_config3(args, dev, ceiling):
    """n = 2^27 lognormal(20, 2) keys saturated to 32 bits (seed 103); 255
    splitters at the quantiles of a 2^16-key sample (seed 1031); the learned
    model is fitted on the GPU from 2^20 keys (seed 1032).  The same
    multisplit runs with the learned identifier and with binary search."""
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    n, m = 1 << 27, 256
    keys = inputs.lognormal_u32(103, n)
    spl = inputs.quantile_splitters(inputs.lognormal_u32(1031, 1 << 16), m)
    fit = inputs.lognormal_u32(1032, 1 << 20)
    dk, _ = keys_device(keys, None, dev)
    ds = torch.from_numpy(spl.view(np.int32)).to(dev)
    dfit = torch.from_numpy(fit.view(np.int32)).to(dev)
    model = torch.empty(ms.MODEL_FLOATS, dtype=torch.float32, device=dev)
    fws = torch.empty(max(256, ms.workspace_size(ms.OP_LEARNED_FIT, len(fit), m)),
                      dtype=torch.uint8, device=dev)
    ev = HipEvents(2)
    for _ in range(3):
        ms.learned_fit(dfit, ds, m, model=model, ws=fws)
    torch.cuda.synchronize()
    ev.record(0)
    reps = 10
    for _ in range(reps):
        ms.learned_fit(dfit, ds, m, model=model, ws=fws)
    ev.record(1)
    torch.cuda.synchronize()
    fit_ms = ev.ms(0, 1) / reps
    ev.close()
    res = {}
    for name, fn in (("learned", ms.BucketFn.learned(ds, model)),
                     ("binary_search", ms.BucketFn.splitter(ds))):
        res[name] = multisplit_row(
            args, "range_2e27_m256_" + name, dk, None, m, fn, ceiling=ceiling, tune=True,
            keep_ids=args.keep_ids, shape=(args.reorder, args.waves, args.items),
            cpu=(lambda: cpu_baseline("range", keys, None, m, 0, args.row_cpu_seconds, 1 << 22,
                                      splitters=spl)) if name == "learned" else None)
    miss = torch.zeros(1, dtype=torch.int64, device=dev)
    ms.keys(dk, m, ms.BucketFn.learned(ds, model), options=ms.Options(mispredicts=miss))
    torch.cuda.synchronize()
    row = res["learned"]
    row["workload"] = "range_2e27_m256"
    row["bucket"] = "learned range (255 lognormal quantile splitters)"
    row["binary_search"] = res["binary_search"]
    row["learned_speedup"] = round(res["binary_search"]["ms_per_call"] / row["ms_per_call"], 4)
    row["learned_beats_binary_search"] = row["value"] > res["binary_search"]["value"]
    row["mispredict_rate"] = round(int(miss.item()) / n, 5)
    row["fit_ms"] = round(fit_ms, 4)
    row["fit_sample"] = len(fit)
    return row


def row_config4(args, dev):
    """4096 independent key-value instances, sizes log-uniform in [2^8, 2^20]
    (seed 104), keys uniform (seed 104000 + i), values = index within the
    instance, m = 64, f(k) = (k >> 8) & 63; tuning from the autotuner; the
    call is captured in a HIP graph and the replays are timed."""
    import numpy as np
    import torch

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs, tuning
    num, m, seed = 4096, 64, 104
    sizes = inputs.batched_sizes(seed, num)
    seg = inputs.segment_offsets(sizes)
    keys, vals = inputs.batched_pairs(seed, sizes)
    total = len(keys)
    dk, dv = keys_device(keys, vals, dev)
    ds = torch.from_numpy(seg.astype(np.int64)).to(dev)
    fn = ms.BucketFn.shift_mask(8, m - 1)
    if args.reorder or args.waves or args.items or args.claim:
        opt = ms.Options(reorder=args.reorder, waves_per_block=args.waves,
                         items_per_lane=args.items, batch_claim=args.claim)
        tune = {"source": "command line"}
    else:
        opt, tune = tuning.tuned_options(ms.OP_BATCHED, dk, dv, m, fn=fn, seg=ds)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    off = torch.empty(num * (m + 1), dtype=torch.int32, device=dev)
    need = ms.workspace_size(ms.OP_BATCHED, total, m, num, opt)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def step(ev):
        if ev is not None:
            ev.record(0)
        ms.batched(dk, dv, ds, m, fn, keys_out=ko, vals_out=vo, offsets=off, options=opt, ws=ws)
        if ev is not None:
            ev.record(1)
    t = time_calls(step, args.steps, args.warmup, stages=False, graph=True)
    # the persistent kernel's own time: the call between two events, minus
    # nothing (the set-up kernel is a few microseconds of one workgroup)
    hev = HipEvents(2)
    torch.cuda.synchronize()
    hev.record(0)
    for _ in range(args.steps):
        ms.batched(dk, dv, ds, m, fn, keys_out=ko, vals_out=vo, offsets=off, options=opt, ws=ws)
    hev.record(1)
    torch.cuda.synchronize()
    eager_ms = hev.ms(0, 1) / args.steps
    hev.close()
    status = ms.batched_status(ws)
    call_ms = t["graph_ms"]
    row = {
        "workload": "batched_4096_m64", "instances": num, "n": total, "m": m, "kv": True,
        "value": round(total / (call_ms * 1e-3) / 1e9, 3), "unit": "Gpairs/s",
        "ms_per_call": round(call_ms, 5),
        "timing": "hipgraph replays, %d calls per graph" % GRAPH_CALLS,
        "eager_ms_per_call": round(eager_ms, 5),
        "status": status,
        "tuning": {"reorder": opt.reorder, "waves_per_block": opt.waves_per_block,
                   "items_per_lane": opt.items_per_lane, "batch_claim": opt.batch_claim},
        "tuner": tune,
        "roofline": roofline("batched", "batched_4096_m64", total * BYTES_PER_PAIR, call_ms),
        "whole_call": whole_call(total, True, call_ms),
    }
    row["roofline"]["kernel"] = "batched_kernel (pre-scan and post-scan items; set-up kernel " \
                                "included)"
    progress("batched_4096_m64: %.3f Gpairs/s" % row["value"])
    if not args.no_cpu_baseline:
        import oracle
        k = keys[:1 << 22]
        v = vals[:1 << 22]
        cut = int(np.searchsorted(seg, 1 << 22, side="right")) - 1
        sseg = seg[:cut + 1].astype(np.uint64)
        units = int(sseg[-1])
        rate, reps = _oracle_rate(
            lambda: oracle.batched(k[:units], v[:units], sseg, m, oracle.SHIFT_MASK, shift=8,
                                   mask=m - 1), units, args.row_cpu_seconds)
        row["cpu_baseline"] = {"value": round(rate, 5), "unit": "Gpairs/s", "cores": 1,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": "the first %d instances (%d pairs), %d reps, "
                                         "single-threaded" % (cut, units, reps)}
    return row


def row_config5(args, dev, ceiling, bits=8, kv=True):
    """LSD radix sort of n = 2^28 pairs (keys seed 105, values = index), 8-bit
    digits, 4 multisplit passes of m = 256."""
    from paper_1701_01189_amd import inputs
    n = 1 << 28
    keys = inputs.uniform_u32(105, n)
    vals = inputs.index_values(n) if kv else None
    dk, dv = keys_device(keys, vals, dev)
    name = "radix_%s_2e28" % ("pairs" if kv else "keys") + ("" if bits == 8 else "_b%d" % bits)
    shape = (args.reorder, args.waves, args.items)
    return multisplit_row(args, name, dk, dv, 0, None, shape=shape, ceiling=ceiling,
                          radix_bits=bits, tune=True,
                          cpu=lambda: cpu_baseline("radix", keys, vals, 0, 0,
                                                   args.row_cpu_seconds, 1 << 22))


def headline(args, dev):
    """2^28 key-only m = 32 (the gate configuration), plus every sub-row."""
    from paper_1701_01189_amd import inputs
    ceiling = None if args.no_ceiling else copy_ceiling(dev)
    n, m = 1 << 28, 32
    keys = inputs.uniform_u32(100, n)
    dk, _ = keys_device(keys, None, dev)
    fn, shift = pow2_fn(m)
    head = multisplit_row(args, "keys_2e28_m32", dk, None, m, fn, ceiling=ceiling)
    del dk
    rows = {}
    groups = [g for g in args.rows.split(",") if g]
    if "sweep" in groups:
        rows.update(rows_sweep(args, keys, dev, ceiling, headline=head))
    if "skew" in groups:
        rows.update(rows_skew(args, dev, ceiling))
    if "config1" in groups:
        rows["keys_2e20_m8"] = row_config1(args, dev, ceiling)
    if "config2" in groups:
        rows.update(rows_config2(args, dev, ceiling))
    if "config3" in groups:
        rows["range_2e27_m256"] = row_config3(args, dev, ceiling)
    if "config4" in groups:
        rows["batched_4096_m64"] = row_config4(args, dev)
    if "config5" in groups:
        rows["radix_pairs_2e28"] = row_config5(args, dev, ceiling)
    gate_rows = {k: r for k, r in rows.items()
                 if k.startswith("keys_2e28_m") and int(k.split("_m")[1]) <= 32}
    gate_rows.setdefault("keys_2e28_m32", head)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "device_warmup_ms": DEVICE_WARMUP_MS,
        "ms_per_step": head["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "keys_2e28_m32: key-only stable multisplit, n = 2^28 uniform "
                               "u32 keys (seed 100), m = 32, f(k) = k >> 27, back-to-back calls",
                   "n": n, "m": m, "kv": False, "seed": 100,
                   "bucket": "shift_mask (delta buckets of width 2^27)"},
        "timing": head["timing"],
        "stage_ms": head["stage_ms"],
        "roofline": head["roofline"],
        "whole_call": head["whole_call"],
        "gate": {"target": "key-only, n = 2^28, m <= 32: whole call >= 60 % of 8 TB/s at "
                           "12 B/key (>= 400 Gkeys/s), back-to-back calls",
                 "per_m": {k: {"value": r["value"], "frac": r["whole_call"]["frac"],
                               "met": r["whole_call"]["frac"] >= GATE_FRAC}
                           for k, r in sorted(gate_rows.items(),
                                              key=lambda kv: int(kv[0].split("_m")[1]))}},
        "rows": rows,
    }
    if "range_2e27_m256" in rows:
        r = rows["range_2e27_m256"]
        line["learned_vs_binary_search"] = {
            "learned": r["value"], "binary_search": r["binary_search"]["value"],
            "unit": "Gkeys/s", "speedup": r["learned_speedup"],
            "learned_beats_binary_search": r["learned_beats_binary_search"],
            "mispredict_rate": r["mispredict_rate"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline("keys", keys, None, m, shift, args.cpu_seconds)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# single workloads
# ---------------------------------------------------------------------------
def single_line(args, row, extra_config=None):
    line = {
        "metric": METRIC, "value": row["value"], "unit": row["unit"], "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "device_warmup_ms": DEVICE_WARMUP_MS,
        "ms_per_step": row["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": row["workload"], **(extra_config or {})},
    }
    for k, v in row.items():
        if k not in line and k not in ("workload", "ms_per_call"):
            line[k] = v
    print(json.dumps(line), flush=True)


def single_multisplit(args, name, dev):
    import numpy as np

    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import inputs
    shape = (args.reorder, args.waves, args.items)
    ceiling = None if args.no_ceiling else copy_ceiling(dev)
    if name.startswith("radix_"):
        bits = int(name.split("_b")[1]) if "_b" in name else 8
        row = row_config5(args, dev, ceiling, bits=bits, kv=name.startswith("radix_pairs"))
        return single_line(args, row)
    if name.startswith("skew_"):
        _, dist, kind, _size, _m = name.split("_")
        n, m = 1 << 25, 256
        keys = inputs.skewed_bucket_keys(100, n, m, dist)
        vals = inputs.index_values(n) if kind == "pairs" else None
        dk, dv = keys_device(keys, vals, dev)
        row = multisplit_row(args, name, dk, dv, m, ms.BucketFn.shift_mask(24, 255),
                             shape=shape, ceiling=ceiling,
                             cpu=lambda: cpu_baseline(kind, keys, vals, m, 24, args.cpu_seconds,
                                                      1 << 22))
        return single_line(args, row)
    if name.startswith("ident_"):
        # ident_keys_2e25_b5: keys uniform in [0, 2^b), identity buckets
        # f(k) = k, m = 2^b (Section 7.1's sweep)
        parts = name.split("_")
        bits = int(parts[3][1:])
        n, m = 1 << int(parts[2][2:]), 1 << bits
        keys = inputs.uniform_u32(120 + bits, n) & np.uint32(m - 1)
        vals = inputs.index_values(n) if parts[1] == "pairs" else None
        dk, dv = keys_device(keys, vals, dev)
        row = multisplit_row(args, name, dk, dv, m, ms.BucketFn.shift_mask(0, m - 1),
                             shape=shape, ceiling=ceiling,
                             cpu=lambda: cpu_baseline(parts[1], keys, vals, m, 0,
                                                      args.cpu_seconds, 1 << 22))
        return single_line(args, row)
    if name == "keys_2e20_m8":
        return single_line(args, row_config1(args, dev, ceiling))
    if name == "pairs_2e25_m32":
        n = 1 << 25
        keys = inputs.uniform_u32(102, n)
        vals = inputs.index_values(n)
        dk, dv = keys_device(keys, vals, dev)
        row = multisplit_row(args, name, dk, dv, 32, ms.BucketFn.shift_mask(27, 31),
                             shape=shape, ceiling=ceiling,
                             cpu=lambda: cpu_baseline("pairs", keys, vals, 32, 27,
                                                      args.cpu_seconds))
        return single_line(args, row)
    if name.startswith("keys_2e28_m") or name.startswith("pairs_2e28_m"):
        m = int(name.split("_m")[1])
        kv = name.startswith("pairs")
        n = 1 << 28
        keys = inputs.uniform_u32(100, n)
        vals = inputs.index_values(n) if kv else None
        dk, dv = keys_device(keys, vals, dev)
        fn, shift = pow2_fn(m)
        cpu = None
        if shift is not None:
            cpu = lambda: cpu_baseline("pairs" if kv else "keys", keys, vals, m, shift,  # noqa
                                       args.cpu_seconds)
        row = multisplit_row(args, name, dk, dv, m, fn, shape=shape, ceiling=ceiling, cpu=cpu)
        if args.cold_reps > 0:
            # informational: one call at a time after evicting the caches
            import torch
            ok = torch.empty_like(dk)
            ov = torch.empty_like(dv) if kv else None

            def step(_ev):
                if kv:
                    ms.pairs(dk, dv, m, fn, keys_out=ok, vals_out=ov)
                else:
                    ms.keys(dk, m, fn, keys_out=ok)
            row["cold_per_call"] = summary(cold_steps(step, args.cold_reps, dev), n)
        return single_line(args, row)
    raise SystemExit("unknown workload %s" % name)


def bench_hist(args, kind, n, m, shift, seed, dev):
    """Device-wide histogram (Section 7.3) of n uniform 32-bit keys: even bins
    f(k) = k >> (32 - log2 m), or range bins over m-1 sorted random splitters
    (seed 113), as in the paper's Even and Range experiments (2^25 elements,
    m <= 256).  One step = one ms_histogram call (pre-scan, then the
    per-bucket reduction of the subproblems' counts), timed from HIP-graph
    replays."""
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
        o = ms.Options(**base) if ev is None else ms.Options(stage_events=ev, **base)
        ms.histogram(dk, m, fn, hist=hist, options=o, ws=ws)
    t = time_calls(step, args.steps, args.warmup, stages=True, graph=True)
    st = t["stage"]
    value = n / (t["graph_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t["graph_ms"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m,
                   "bins": "range (m-1 random splitters)" if spl is not None else
                           "even (k >> %d)" % shift, "seed": seed, **base},
        "timing": "hipgraph replays, %d calls per graph" % GRAPH_CALLS,
        "eager_value": round(n / (t["ms"] * 1e-3) / 1e9, 3),
        "stage_ms": {"prescan": round(st[0], 5), "reduce": round(st[1], 5)},
        "roofline": roofline("prescan", args.workload, 4.0 * n, st[0]),
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = min(n, 1 << 24)
        if spl is not None:
            run = lambda: oracle.histogram(keys[:sample], m, oracle.SPLITTERS, splitters=spl)  # noqa
        else:
            run = lambda: oracle.histogram(keys[:sample], m, oracle.SHIFT_MASK, shift=shift,  # noqa
                                           mask=m - 1)
        rate, reps = _oracle_rate(run, sample, args.cpu_seconds)
        line["cpu_baseline"] = {"value": rate, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
                                "cpu_model": cpu_model(),
                                "sample": "the first %d keys, %d reps" % (sample, reps)}
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
        rate, reps = _oracle_rate(lambda: oracle.sssp(row, col, wt, 0), ne / 1e3,
                                  args.cpu_seconds, max_reps=20)
        line["cpu_baseline"] = {"value": round(rate * 1e3, 2), "unit": "MTEPS",
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
    for _ in range(args.warmup):
        ms.copy_u32(b, a)
    hev = HipEvents(2)
    torch.cuda.synchronize()
    hev.record(0)
    for _ in range(args.steps):
        ms.copy_u32(b, a)
    hev.record(1)
    torch.cuda.synchronize()
    t = hev.ms(0, 1) / args.steps
    hev.close()
    gbps = 8.0 * n / (t * 1e-3) / 1e9
    print(json.dumps({"metric": "streaming copy GB/s (ceiling probe)", "value": round(gbps, 1),
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(t, 5), "higher_is_better": True, "dtype": "u32",
                      "data": "synthetic", "config": {"workload": "copy_2e28", "n": n,
                                                      "bytes_per_launch": 8 * n}}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the multisplit library runs on one GPU; only --gpus 1 is "
              "measured (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1701_01189_amd import build as b

    if not os.path.exists(b.LIB):
        b.build(force=True)
    dev = torch.device("cuda:0")
    global DEVICE_WARMUP_MS
    DEVICE_WARMUP_MS = args.device_warmup_ms
    w = args.workload
    if w == "headline":
        return headline(args, dev)
    if w == "range_2e27_m256":
        return single_line(args, row_config3(args, dev, None))
    if w == "batched_4096_m64":
        return single_line(args, row_config4(args, dev))
    if w == "copy_2e28":
        return bench_copy(args, 1 << 28, dev)
    if w.startswith("sssp_rmat_2e20"):
        delta = int(w.split("_d")[1]) if "_d" in w else 800
        return bench_sssp(args, 20, 4_800_000, delta, 106, dev)
    if w.startswith("hist_") or w.startswith("histrange_"):
        size, mm = w.split("_")[1], int(w.split("_m")[1])
        return bench_hist(args, w.split("_")[0], 1 << int(size[2:]), mm,
                          32 - (mm - 1).bit_length(), 110, dev)
    return single_multisplit(args, w, dev)


if __name__ == "__main__":
    main()
