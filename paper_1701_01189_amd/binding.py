"""Thin ctypes binding of libmultisplit.so (include/multisplit.h).

Argument marshalling only: torch tensors supply device pointers, the current
HIP stream and workspace memory; every step of the multisplit runs in the
library's gfx950 kernels.  There is no fallback: if the library is missing
or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmultisplit.so")

MS_OK = 0
STATUS = {0: "MS_OK", -1: "MS_ERR_INVALID_ARG", -2: "MS_ERR_WORKSPACE", -3: "MS_ERR_HIP",
          -4: "MS_ERR_BUCKET_RANGE", -5: "MS_ERR_TIMEOUT", -6: "MS_ERR_UNSUPPORTED"}

BUCKET_SHIFT_MASK, BUCKET_DIV, BUCKET_SPLITTERS, BUCKET_LEARNED = 0, 1, 2, 3
REORDER_AUTO, REORDER_BLOCK, REORDER_WAVE, REORDER_NONE = 0, 1, 2, 3
PRESCAN_AUTO, PRESCAN_BALLOT, PRESCAN_LANES = 0, 1, 2
OP_KEYS, OP_PAIRS, OP_BATCHED, OP_RADIX_SORT, OP_RADIX_SORT_PAIRS, OP_LEARNED_FIT, OP_HISTOGRAM = \
    range(7)
MODEL_LEAVES = 256
MODEL_FLOATS = 2 + 2 * MODEL_LEAVES


class MultisplitError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))
        self.status = status


class BucketFnC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("shift", ctypes.c_uint32), ("mask", ctypes.c_uint32),
                ("divisor", ctypes.c_uint32), ("splitters", ctypes.c_void_p),
                ("model", ctypes.c_void_p)]


class SsspStatsC(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("items_split", ctypes.c_uint64),
                ("edges_relaxed", ctypes.c_uint64), ("pushes", ctypes.c_uint64),
                ("max_pending", ctypes.c_uint64)]


class OptionsC(ctypes.Structure):
    _fields_ = [("reorder", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("items_per_lane", ctypes.c_int32), ("max_chunks", ctypes.c_int32),
                ("stage_events", ctypes.c_void_p), ("d_mispredicts", ctypes.c_void_p),
                ("batch_claim", ctypes.c_uint32), ("spin_limit", ctypes.c_uint32),
                ("test_flags", ctypes.c_uint32), ("prescan", ctypes.c_int32),
                ("keep_bucket_ids", ctypes.c_int32)]


_lib = None
SYMBOLS = ["ms_status_str", "ms_version", "ms_workspace_size", "ms_keys", "ms_pairs",
           "ms_pairs_noalloc",
           "ms_radix_sort", "ms_batched", "ms_batched_status", "ms_learned_fit", "ms_copy_u32",
           "ms_autotune", "ms_sssp", "ms_sssp_workspace_size"]


def lib():
    """Loads libmultisplit.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmultisplit.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1701_01189_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u32, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int
    L.ms_status_str.argtypes = [i32]
    L.ms_status_str.restype = ctypes.c_char_p
    L.ms_version.argtypes = []
    L.ms_version.restype = ctypes.c_char_p
    L.ms_workspace_size.argtypes = [i32, sz, u32, u32, ctypes.POINTER(OptionsC)]
    L.ms_workspace_size.restype = sz
    L.ms_keys.argtypes = [vp, vp, vp, sz, u32, ctypes.POINTER(BucketFnC), vp, sz,
                          ctypes.POINTER(OptionsC), vp]
    L.ms_keys.restype = i32
    L.ms_pairs.argtypes = [vp, vp, vp, vp, vp, sz, u32, ctypes.POINTER(BucketFnC), vp, sz,
                           ctypes.POINTER(OptionsC), vp]
    L.ms_pairs.restype = i32
    L.ms_pairs_noalloc.argtypes = [vp, vp, vp, vp, vp, sz, u32, ctypes.POINTER(BucketFnC),
                                   ctypes.POINTER(OptionsC), vp]
    L.ms_pairs_noalloc.restype = i32
    L.ms_histogram.argtypes = [vp, sz, u32, ctypes.POINTER(BucketFnC), vp, vp, sz,
                               ctypes.POINTER(OptionsC), vp]
    L.ms_histogram.restype = i32
    L.ms_radix_sort.argtypes = [vp, vp, vp, vp, sz, u32, vp, sz, ctypes.POINTER(OptionsC), vp]
    L.ms_radix_sort.restype = i32
    L.ms_batched.argtypes = [vp, vp, vp, vp, vp, u32, sz, u32, ctypes.POINTER(BucketFnC), vp, vp,
                             sz, ctypes.POINTER(OptionsC), vp]
    L.ms_batched.restype = i32
    L.ms_autotune.argtypes = [i32, vp, vp, vp, vp, vp, u32, sz, u32, ctypes.POINTER(BucketFnC),
                              vp, sz, i32, ctypes.POINTER(OptionsC), ctypes.POINTER(OptionsC),
                              ctypes.POINTER(ctypes.c_float), vp]
    L.ms_autotune.restype = i32
    L.ms_batched_status.argtypes = [vp, vp]
    L.ms_batched_status.restype = i32
    L.ms_learned_fit.argtypes = [vp, vp, sz, vp, u32, vp, vp, sz, vp]
    L.ms_learned_fit.restype = i32
    L.ms_copy_u32.argtypes = [vp, vp, sz, vp]
    L.ms_copy_u32.restype = i32
    u64 = ctypes.c_uint64
    L.ms_sssp_workspace_size.argtypes = [u32, u64, u32]
    L.ms_sssp_workspace_size.restype = sz
    L.ms_sssp.argtypes = [vp, vp, vp, u32, u64, u32, u32, u32, vp, vp, sz,
                          ctypes.POINTER(SsspStatsC), vp]
    L.ms_sssp.restype = i32
    _lib = L
    return L


def _check(rc, what):
    if rc != MS_OK:
        raise MultisplitError(rc, what)


def _ptr(t):
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _u32(t, name):
    if t is None:
        return None
    if t.element_size() != 4:
        raise ValueError("%s must hold 32-bit elements" % name)
    return _ptr(t)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class BucketFn:
    """Bucket identifier descriptor (MS_BUCKET_*)."""

    def __init__(self, kind, shift=0, mask=0, divisor=0, splitters=None, model=None):
        self.kind, self.shift, self.mask, self.divisor = kind, shift, mask, divisor
        self.splitters, self.model = splitters, model

    @staticmethod
    def shift_mask(shift, mask):
        return BucketFn(BUCKET_SHIFT_MASK, shift=shift, mask=mask)

    @staticmethod
    def div(divisor):
        return BucketFn(BUCKET_DIV, divisor=divisor)

    @staticmethod
    def splitter(splitters):
        return BucketFn(BUCKET_SPLITTERS, splitters=splitters)

    @staticmethod
    def learned(splitters, model):
        return BucketFn(BUCKET_LEARNED, splitters=splitters, model=model)

    def c(self):
        return BucketFnC(self.kind, self.shift, self.mask, self.divisor,
                         _u32(self.splitters, "splitters"),
                         _ptr(self.model) if self.model is not None else None)


class Options:
    """Tuning and instrumentation (ms_options); all fields optional."""

    def __init__(self, reorder=0, waves_per_block=0, items_per_lane=0, max_chunks=0,
                 stage_events=None, mispredicts=None, batch_claim=0, spin_limit=0,
                 test_flags=0, prescan=0, keep_bucket_ids=0):
        self.reorder, self.waves_per_block = reorder, waves_per_block
        self.prescan, self.keep_bucket_ids = prescan, keep_bucket_ids
        self.items_per_lane, self.max_chunks = items_per_lane, max_chunks
        self.batch_claim, self.spin_limit, self.test_flags = batch_claim, spin_limit, test_flags
        self.stage_events = stage_events   # list of 4 torch.cuda.Event or None
        self.mispredicts = mispredicts     # 1-element int64 CUDA tensor or None
        self._ev = None

    def c(self):
        ev = None
        if self.stage_events is not None:
            self._ev = (ctypes.c_void_p * 4)(*[e.cuda_event for e in self.stage_events])
            ev = ctypes.cast(self._ev, ctypes.c_void_p)
        return OptionsC(self.reorder, self.waves_per_block, self.items_per_lane,
                        self.max_chunks, ev, _ptr(self.mispredicts), self.batch_claim,
                        self.spin_limit, self.test_flags, self.prescan, self.keep_bucket_ids)


def _opt(options):
    return ctypes.byref(options.c()) if options is not None else None


def workspace_size(op, n, m, num_inst=0, options=None):
    return int(lib().ms_workspace_size(op, n, m, num_inst, _opt(options)))


def _workspace(op, n, m, device, options=None, num_inst=0, ws=None):
    import torch
    need = workspace_size(op, n, m, num_inst, options)
    if need == 0 and n > 0:
        raise MultisplitError(-1, "ms_workspace_size")
    if ws is not None:
        return ws, ws.numel() * ws.element_size()
    return torch.empty(max(need, 256), dtype=torch.uint8, device=device), max(need, 256)


def keys(keys_in, m, fn, keys_out=None, offsets=None, options=None, stream=None, ws=None):
    """Stable multisplit of a 32-bit key tensor.  Returns (keys_out, offsets)."""
    import torch
    n = keys_in.numel()
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    if offsets is None:
        offsets = torch.empty(m + 1, dtype=torch.int32, device=keys_in.device)
    w, wb = _workspace(OP_KEYS, n, m, keys_in.device, options, ws=ws)
    f = fn.c()
    o = options.c() if options is not None else None
    rc = lib().ms_keys(_u32(keys_in, "keys_in"), _u32(keys_out, "keys_out"),
                       _u32(offsets, "offsets"), n, m, ctypes.byref(f), _ptr(w), wb,
                       ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "ms_keys")
    return keys_out, offsets


def pairs(keys_in, vals_in, m, fn, keys_out=None, vals_out=None, offsets=None, options=None,
          stream=None, ws=None):
    """Stable multisplit of key-value pairs.  Returns (keys_out, vals_out, offsets)."""
    import torch
    n = keys_in.numel()
    if vals_in.numel() != n:
        raise ValueError("keys and values differ in length")
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    if vals_out is None:
        vals_out = torch.empty_like(vals_in)
    if offsets is None:
        offsets = torch.empty(m + 1, dtype=torch.int32, device=keys_in.device)
    w, wb = _workspace(OP_PAIRS, n, m, keys_in.device, options, ws=ws)
    f = fn.c()
    o = options.c() if options is not None else None
    rc = lib().ms_pairs(_u32(keys_in, "keys_in"), _u32(vals_in, "vals_in"),
                        _u32(keys_out, "keys_out"), _u32(vals_out, "vals_out"),
                        _u32(offsets, "offsets"), n, m, ctypes.byref(f), _ptr(w), wb,
                        ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "ms_pairs")
    return keys_out, vals_out, offsets


def pairs_noalloc(keys_in, vals_in, m, fn, keys_out, vals_out, offsets, options=None,
                  stream=None):
    """ms_pairs_noalloc: the stable multisplit without a workspace (the
    library's static device array serves).  vals_in / vals_out None: key
    only.  The caller passes every output; nothing is allocated."""
    n = keys_in.numel()
    if vals_in is not None and vals_in.numel() != n:
        raise ValueError("keys and values differ in length")
    f = fn.c()
    o = options.c() if options is not None else None
    rc = lib().ms_pairs_noalloc(_u32(keys_in, "keys_in"),
                                _u32(vals_in, "vals_in") if vals_in is not None else None,
                                _u32(keys_out, "keys_out"),
                                _u32(vals_out, "vals_out") if vals_out is not None else None,
                                _u32(offsets, "offsets") if offsets is not None else None,
                                n, m, ctypes.byref(f),
                                ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "ms_pairs_noalloc")
    return keys_out, vals_out, offsets


def histogram(keys_in, m, fn, hist=None, options=None, stream=None, ws=None):
    """Device-wide histogram of fn over a 32-bit key tensor: hist[j] = number
    of keys in bucket j.  Returns hist (m int32, read as uint32)."""
    import torch
    n = keys_in.numel()
    if hist is None:
        hist = torch.empty(m, dtype=torch.int32, device=keys_in.device)
    w, wb = _workspace(OP_HISTOGRAM, n, m, keys_in.device, options, ws=ws)
    f = fn.c()
    o = options.c() if options is not None else None
    rc = lib().ms_histogram(_u32(keys_in, "keys_in"), n, m, ctypes.byref(f), _u32(hist, "hist"),
                            _ptr(w), wb, ctypes.byref(o) if o is not None else None,
                            _stream(stream))
    _check(rc, "ms_histogram")
    return hist


def radix_sort(keys_in, vals_in=None, bits_per_pass=8, keys_out=None, vals_out=None,
               options=None, stream=None, ws=None):
    """LSD radix sort from multisplit passes.  Returns (keys_out, vals_out or None)."""
    import torch
    n = keys_in.numel()
    kv = vals_in is not None
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    if kv and vals_out is None:
        vals_out = torch.empty_like(vals_in)
    w, wb = _workspace(OP_RADIX_SORT_PAIRS if kv else OP_RADIX_SORT, n, 1 << bits_per_pass,
                       keys_in.device, options, ws=ws)
    o = options.c() if options is not None else None
    rc = lib().ms_radix_sort(_u32(keys_in, "keys_in"), _u32(vals_in, "vals_in"),
                             _u32(keys_out, "keys_out"), _u32(vals_out, "vals_out"), n,
                             bits_per_pass, _ptr(w), wb,
                             ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "ms_radix_sort")
    return keys_out, vals_out


def batched(keys_in, vals_in, seg, m, fn, keys_out=None, vals_out=None, offsets=None,
            options=None, stream=None, ws=None):
    """Batched multisplit of the instances [seg[i], seg[i+1]) of the
    concatenated inputs.  seg: int64 CUDA tensor of num+1 offsets.  Returns
    (keys_out, vals_out or None, offsets[num*(m+1)], workspace)."""
    import torch
    n = keys_in.numel()
    num = seg.numel() - 1
    kv = vals_in is not None
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    if kv and vals_out is None:
        vals_out = torch.empty_like(vals_in)
    if offsets is None:
        offsets = torch.empty(max(1, num * (m + 1)), dtype=torch.int32, device=keys_in.device)
    if seg.element_size() != 8:
        raise ValueError("seg must hold 64-bit offsets")
    w, wb = _workspace(OP_BATCHED, n, m, keys_in.device, options, num_inst=num, ws=ws)
    f = fn.c()
    o = options.c() if options is not None else None
    rc = lib().ms_batched(_u32(keys_in, "keys_in"), _u32(vals_in, "vals_in"),
                          _u32(keys_out, "keys_out"), _u32(vals_out, "vals_out"), _ptr(seg),
                          num, n, m, ctypes.byref(f), _u32(offsets, "offsets"), _ptr(w), wb,
                          ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "ms_batched")
    return keys_out, vals_out, offsets, w


def autotune(op, keys_in, vals_in, m, fn=None, seg=None, reps=3, base=None, stream=None):
    """Times every candidate tuning of `op` on these inputs (scratch outputs
    and workspace are allocated here) and returns (Options, milliseconds)."""
    import torch
    n = keys_in.numel()
    num = seg.numel() - 1 if seg is not None else 0
    ko = torch.empty_like(keys_in)
    vo = torch.empty_like(vals_in) if vals_in is not None else None
    radix = op in (OP_RADIX_SORT, OP_RADIX_SORT_PAIRS)
    need = 0
    # the workspace of the largest candidate (ms_autotune's lists; a shape
    # the operation does not have sizes to 0)
    shapes = ((8, 8, 1), (8, 4, 1), (4, 8, 1), (4, 16, 1), (16, 8, 1), (16, 16, 1), (8, 8, 2),
              (4, 16, 2), (8, 8, 3))
    if op == OP_BATCHED:
        shapes = ((8, 8, 1), (8, 4, 1), (4, 16, 1), (4, 8, 1), (16, 4, 1), (16, 8, 1))
    keep = base.keep_bucket_ids if base is not None else 0
    for wpb, nw, mode in shapes:
        need = max(need, workspace_size(op, n, (1 << m) if radix else m, num,
                                        Options(reorder=mode, waves_per_block=wpb,
                                                items_per_lane=nw, keep_bucket_ids=keep)))
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=keys_in.device)
    best = OptionsC()
    ms_ = ctypes.c_float(0.0)
    f = fn.c() if fn is not None else BucketFnC(0, 0, 0, 0, None, None)
    b = base.c() if base is not None else None
    rc = lib().ms_autotune(op, _u32(keys_in, "keys_in"), _u32(vals_in, "vals_in"), _u32(ko, "ko"),
                           _u32(vo, "vo"), _ptr(seg) if seg is not None else None, num, n, m,
                           ctypes.byref(f), _ptr(ws), ws.numel(), reps,
                           ctypes.byref(b) if b is not None else None, ctypes.byref(best),
                           ctypes.byref(ms_), _stream(stream))
    _check(rc, "ms_autotune")
    opt = Options(reorder=best.reorder, waves_per_block=best.waves_per_block,
                  items_per_lane=best.items_per_lane, max_chunks=best.max_chunks,
                  batch_claim=best.batch_claim, spin_limit=best.spin_limit,
                  test_flags=best.test_flags, prescan=best.prescan,
                  keep_bucket_ids=best.keep_bucket_ids)
    return opt, float(ms_.value)


def batched_status(ws, stream=None):
    """MS_OK or MS_ERR_TIMEOUT for the last batched call on workspace ws."""
    return int(lib().ms_batched_status(_ptr(ws), _stream(stream)))


def learned_fit(sample, splitters, m, model=None, labels=None, stream=None, ws=None):
    """Fits the two-stage learned bucket model on the GPU, to the upper-bound
    bucket ids over the splitters or to the given labels.  Returns the model
    tensor (MODEL_FLOATS float32)."""
    import torch
    if model is None:
        model = torch.empty(MODEL_FLOATS, dtype=torch.float32, device=sample.device)
    n = sample.numel()
    if labels is not None and labels.numel() != n:
        raise ValueError("labels and sample differ in length")
    if ws is None:
        need = workspace_size(OP_LEARNED_FIT, n, m)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=sample.device)
    rc = lib().ms_learned_fit(_u32(sample, "sample"), _u32(labels, "labels"), n,
                              _u32(splitters, "splitters"), m, _ptr(model), _ptr(ws),
                              ws.numel(), _stream(stream))
    _check(rc, "ms_learned_fit")
    return model


def copy_u32(dst, src, stream=None):
    rc = lib().ms_copy_u32(_u32(dst, "dst"), _u32(src, "src"), src.numel(), _stream(stream))
    _check(rc, "ms_copy_u32")
    return dst


INF = 0xFFFFFFFF


def sssp_workspace_size(nv, ne, num_buckets=10):
    return int(lib().ms_sssp_workspace_size(nv, ne, num_buckets))


def sssp(row, col, wt, source, delta=100, num_buckets=10, dist=None, ws=None, stream=None):
    """Shortest-path distances from `source` by delta-stepping with multisplit
    bucketing.  row: int64 tensor of nv + 1 CSR offsets; col, wt: 32-bit
    tensors of ne targets and weights (all on the GPU).  Returns (dist, stats):
    dist an int32 tensor holding the uint32 distances (INF where unreachable),
    stats a dict of round counts."""
    import torch
    if row.dtype != torch.int64:
        raise ValueError("row must hold 64-bit offsets")
    nv, ne = row.numel() - 1, col.numel()
    if wt.numel() != ne:
        raise ValueError("col and wt differ in length")
    if dist is None:
        dist = torch.empty(max(nv, 1), dtype=torch.int32, device=row.device)
    if ws is None:
        need = sssp_workspace_size(nv, ne, num_buckets)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=row.device)
    st = SsspStatsC()
    rc = lib().ms_sssp(_ptr(row), _u32(col, "col") if ne else None,
                       _u32(wt, "wt") if ne else None, nv, ne, source, delta, num_buckets,
                       _u32(dist, "dist"), _ptr(ws), ws.numel(), ctypes.byref(st),
                       _stream(stream))
    _check(rc, "ms_sssp")
    return dist, {k: int(getattr(st, k)) for k, _ in SsspStatsC._fields_}
