"""CPU oracle for stable multisplit -- TEST INFRASTRUCTURE, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU path never calls it, and it
shares no code with the GPU path (it has its own C++ source, built with g++).

Each function restates a definition from the paper (Ashkiani et al., "GPU
Multisplit: an extended study of a parallel algorithm"): the stable multisplit
of Section 3.1 / Eq. (1), the bucket identifiers of Section 6, the radix sort
of Section 7.1, and the shortest-path distances that the delta-stepping of
Section 7.2 computes (Dijkstra's algorithm).  See ``oracle.cpp`` for the per-function citations.

Bucket kinds use the oracle's own numbering:
    SHIFT_MASK (0): (k >> p0) & p1
    DIV        (1): k // p0
    SPLITTERS  (2): number of splitters <= k (upper bound over m-1 splitters)
    LEARNED    (3): same ids as SPLITTERS (the learned model must match them)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

SHIFT_MASK, DIV, SPLITTERS, LEARNED = 0, 1, 2, 3
LEAVES = 256

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compiles the oracle with g++ (no HIP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if a is not None else None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    P32 = ctypes.POINTER(ctypes.c_uint32)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    PF = ctypes.POINTER(ctypes.c_float)
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.or_bucket_ids.argtypes = [P32, u64, u32, i32, u32, u32, P32, P32]
    lib.or_bucket_ids.restype = i32
    lib.or_histogram.argtypes = [P32, u64, u32, i32, u32, u32, P32, P32]
    lib.or_histogram.restype = i32
    lib.or_multisplit.argtypes = [P32, P32, u64, u32, i32, u32, u32, P32, P32, P32, P32]
    lib.or_multisplit.restype = i32
    lib.or_radix_sort.argtypes = [P32, P32, u64, P32, P32]
    lib.or_radix_sort.restype = None
    lib.or_batched.argtypes = [P32, P32, P64, u32, u32, i32, u32, u32, P32, P32, P32, P32]
    lib.or_batched.restype = i32
    lib.or_learned_leaf.argtypes = [PF, u32]
    lib.or_learned_leaf.restype = u32
    lib.or_learned_predict.argtypes = [PF, u32, u32]
    lib.or_learned_predict.restype = u32
    lib.or_learned_fit.argtypes = [P32, u64, P32, u32, P32, PF]
    lib.or_learned_fit.restype = None
    lib.or_learned_bucket_ids.argtypes = [PF, P32, u32, P32, u64, P32, P64]
    lib.or_learned_bucket_ids.restype = None
    lib.or_sssp.argtypes = [P64, P32, P32, u32, u32, P32]
    lib.or_sssp.restype = i32
    _lib = lib
    return lib


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _params(kind, shift=0, mask=0, divisor=0):
    if kind == SHIFT_MASK:
        return shift, mask
    if kind == DIV:
        return divisor, 0
    return 0, 0


def bucket_ids(keys, m, kind, shift=0, mask=0, divisor=0, splitters=None):
    keys = _c32(keys)
    out = np.empty(len(keys), dtype=np.uint32)
    spl = _c32(splitters) if splitters is not None else None
    p0, p1 = _params(kind, shift, mask, divisor)
    rc = _load().or_bucket_ids(_u32p(keys), len(keys), m, kind, p0, p1, _u32p(spl), _u32p(out))
    if rc:
        raise ValueError("bucket id outside [0, m)")
    return out


def histogram(keys, m, kind, shift=0, mask=0, divisor=0, splitters=None):
    """Section 7.3: number of keys per bucket (m uint32)."""
    keys = _c32(keys)
    out = np.empty(m, dtype=np.uint32)
    spl = _c32(splitters) if splitters is not None else None
    p0, p1 = _params(kind, shift, mask, divisor)
    rc = _load().or_histogram(_u32p(keys), len(keys), m, kind, p0, p1, _u32p(spl), _u32p(out))
    if rc:
        raise ValueError("bucket id outside [0, m)")
    return out


def multisplit(keys, m, kind, vals=None, shift=0, mask=0, divisor=0, splitters=None):
    """Returns (out_keys, out_vals or None, offsets[m+1])."""
    keys = _c32(keys)
    n = len(keys)
    vals = _c32(vals) if vals is not None else None
    spl = _c32(splitters) if splitters is not None else None
    ok = np.empty(n, dtype=np.uint32)
    ov = np.empty(n, dtype=np.uint32) if vals is not None else None
    off = np.empty(m + 1, dtype=np.uint32)
    p0, p1 = _params(kind, shift, mask, divisor)
    rc = _load().or_multisplit(_u32p(keys), _u32p(vals), n, m, kind, p0, p1, _u32p(spl),
                               _u32p(ok), _u32p(ov), _u32p(off))
    if rc:
        raise ValueError("bucket id outside [0, m)")
    return ok, ov, off


def radix_sort(keys, vals=None):
    keys = _c32(keys)
    n = len(keys)
    vals = _c32(vals) if vals is not None else None
    ok = np.empty(n, dtype=np.uint32)
    ov = np.empty(n, dtype=np.uint32) if vals is not None else None
    _load().or_radix_sort(_u32p(keys), _u32p(vals), n, _u32p(ok), _u32p(ov))
    return ok, ov


def batched(keys, vals, seg, m, kind, shift=0, mask=0, divisor=0, splitters=None):
    keys = _c32(keys)
    vals = _c32(vals) if vals is not None else None
    seg = np.ascontiguousarray(seg, dtype=np.uint64)
    num = len(seg) - 1
    spl = _c32(splitters) if splitters is not None else None
    ok = np.empty(len(keys), dtype=np.uint32)
    ov = np.empty(len(keys), dtype=np.uint32) if vals is not None else None
    off = np.empty(num * (m + 1), dtype=np.uint32)
    p0, p1 = _params(kind, shift, mask, divisor)
    rc = _load().or_batched(_u32p(keys), _u32p(vals),
                            seg.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), num, m, kind,
                            p0, p1, _u32p(spl), _u32p(ok), _u32p(ov), _u32p(off))
    if rc:
        raise ValueError("bucket id outside [0, m)")
    return ok, ov, off


def _fp(model):
    return model.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def learned_fit(sample, splitters, m, labels=None):
    """The model fitted to sample keys labelled by the upper bound over the
    splitters, or by `labels` (clamped to m - 1) when given."""
    sample = _c32(sample)
    spl = _c32(splitters)
    lab = _c32(labels) if labels is not None else None
    model = np.zeros(2 + 2 * LEAVES, dtype=np.float32)
    _load().or_learned_fit(_u32p(sample), len(sample), _u32p(spl), m, _u32p(lab), _fp(model))
    return model


def learned_leaf(model, k):
    model = np.ascontiguousarray(model, dtype=np.float32)
    return int(_load().or_learned_leaf(_fp(model), int(k)))


def learned_predict(model, m, k):
    model = np.ascontiguousarray(model, dtype=np.float32)
    return int(_load().or_learned_predict(_fp(model), m, int(k)))


def learned_bucket_ids(model, splitters, m, keys):
    """Returns (exact ids, number of raw-model mispredictions)."""
    model = np.ascontiguousarray(model, dtype=np.float32)
    spl = _c32(splitters)
    keys = _c32(keys)
    out = np.empty(len(keys), dtype=np.uint32)
    miss = ctypes.c_uint64(0)
    _load().or_learned_bucket_ids(_fp(model), _u32p(spl), m, _u32p(keys), len(keys),
                                  _u32p(out), ctypes.byref(miss))
    return out, int(miss.value)


INF = 0xFFFFFFFF


def sssp(row, col, wt, src):
    """Shortest-path distances from src over a CSR graph (row: nv+1 offsets,
    col/wt: one entry per directed edge); INF where unreachable."""
    row = np.ascontiguousarray(row, dtype=np.uint64)
    col, wt = _c32(col), _c32(wt)
    nv = len(row) - 1
    dist = np.empty(nv, dtype=np.uint32)
    rc = _load().or_sssp(row.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _u32p(col),
                         _u32p(wt), nv, int(src), _u32p(dist))
    if rc != 0:
        raise ValueError("a shortest path does not fit in 32 bits")
    return dist
