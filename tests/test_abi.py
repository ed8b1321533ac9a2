"""The C ABI library loads, exports every declared symbol, and rejects invalid
arguments on the host before touching a GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "multisplit.h")


@pytest.fixture(scope="module")
def L():
    from paper_1701_01189_amd import binding, build
    if build.stale():
        build.build(force=True)
    return binding.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "ms_keys" in names and "ms_pairs" in names and "ms_radix_sort" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    assert L.ms_status_str(0) == b"MS_OK"
    assert L.ms_status_str(-2) == b"MS_ERR_WORKSPACE"
    assert L.ms_version().startswith(b"multisplit")


def fake(addr):
    return ctypes.c_void_p(addr)


def test_host_validation_rejects_before_launch(L):
    from paper_1701_01189_amd.binding import BucketFnC, OptionsC
    fn = BucketFnC(0, 27, 31, 0, None, None)
    ki, ko, ws = fake(0x1000000), fake(0x9000000), fake(0x20000000)
    n = 1000
    need = L.ms_workspace_size(0, n, 32, 0, None)
    assert need > 0
    # m out of range
    assert L.ms_keys(ki, ko, None, n, 0, ctypes.byref(fn), ws, need, None, None) == -1
    assert L.ms_keys(ki, ko, None, n, 65537, ctypes.byref(fn), ws, need, None, None) == -1
    # null pointers with n > 0, and overlapping in/out
    assert L.ms_keys(None, ko, None, n, 32, ctypes.byref(fn), ws, need, None, None) == -1
    assert L.ms_keys(ki, fake(0x1000000 + 8), None, n, 32, ctypes.byref(fn), ws, need, None,
                     None) == -1
    # n >= 2^32 - 1
    assert L.ms_keys(ki, ko, None, 2**32, 32, ctypes.byref(fn), ws, need, None, None) == -1
    # bucket function that can reach m or beyond
    bad = BucketFnC(0, 27, 63, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(bad), ws, need, None, None) == -4
    bad = BucketFnC(1, 0, 0, 1000, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(bad), ws, need, None, None) == -4
    bad = BucketFnC(2, 0, 0, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(bad), ws, need, None, None) == -1
    bad = BucketFnC(7, 0, 0, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(bad), ws, need, None, None) == -1
    # workspace too small or missing
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), ws, need - 1, None, None) == -2
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), None, need, None, None) == -2
    # unsupported shape and bad options
    o = OptionsC(1, 6, 8, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), ws, need, ctypes.byref(o), None) == -6
    o = OptionsC(9, 0, 0, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), ws, need, ctypes.byref(o), None) == -1
    # pre-scan method: out of range, and lane counters without block reordering
    o = OptionsC(0, 0, 0, 0, None, None, 0, 0, 0, 3)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), ws, need, ctypes.byref(o), None) == -1
    o = OptionsC(2, 8, 8, 0, None, None, 0, 0, 0, 2)
    assert L.ms_keys(ki, ko, None, n, 32, ctypes.byref(fn), ws, need, ctypes.byref(o), None) == -6
    # pairs: values missing on one side
    assert L.ms_pairs(ki, None, ko, fake(0x30000000), None, n, 32, ctypes.byref(fn), ws, need,
                      None, None) == -1
    # histogram: missing or overlapping output, bad m, small workspace, bad bucket function
    hh = fake(0x40000000)
    assert L.ms_histogram(ki, n, 32, ctypes.byref(fn), None, ws, need, None, None) == -1
    assert L.ms_histogram(ki, n, 0, ctypes.byref(fn), hh, ws, need, None, None) == -1
    assert L.ms_histogram(ki, n, 32, ctypes.byref(fn), fake(0x1000000 + 64), ws, need, None,
                          None) == -1
    assert L.ms_histogram(ki, n, 32, ctypes.byref(fn), fake(0x1000000 - 64), ws, need, None,
                          None) == -1
    assert L.ms_histogram(ki, n, 32, ctypes.byref(fn), hh, ws, need - 1, None, None) == -2
    bad = BucketFnC(0, 27, 63, 0, None, None)
    assert L.ms_histogram(ki, n, 32, ctypes.byref(bad), hh, ws, need, None, None) == -4
    assert L.ms_workspace_size(6, n, 32, 0, None) == need
    # radix sort: bits per pass out of range
    assert L.ms_radix_sort(ki, None, ko, None, n, 9, ws, 1 << 30, None, None) == -1
    assert L.ms_radix_sort(ki, None, ko, None, n, 0, ws, 1 << 30, None, None) == -1


def test_workspace_sizes(L):
    from paper_1701_01189_amd.binding import OptionsC
    a = L.ms_workspace_size(0, 1 << 20, 8, 0, None)
    b = L.ms_workspace_size(0, 1 << 28, 256, 0, None)
    assert 0 < a < b
    assert b < 8 << 20  # H stays small: m x L0 words
    r = L.ms_workspace_size(4, 1 << 28, 256, 0, None)
    assert r >= 2 * 4 * (1 << 28)  # ping-pong keys and values
    assert L.ms_workspace_size(0, 1000, 0, 0, None) == 0
    o = OptionsC(2, 8, 8, 0, None, None)
    assert L.ms_workspace_size(1, 1 << 25, 32, 0, ctypes.byref(o)) > 0


def test_default_shape_for_every_reorder_mode(L):
    """Only the reordering mode set: the library picks a supported tile shape
    for every m (a wave-level or direct call at m > 64 must not inherit the
    block-level 16 x 8 default)."""
    from paper_1701_01189_amd.binding import OptionsC
    for mode in (0, 1, 2, 3):
        for m in (1, 2, 32, 64, 65, 200, 256):
            o = OptionsC(mode, 0, 0, 0, None, None)
            for op in (0, 1, 6):
                assert L.ms_workspace_size(op, 1 << 20, m, 0, ctypes.byref(o)) > 0, (mode, m, op)


def test_more_than_256_buckets_host_checks(L):
    """m up to 65536 for shift/mask and delta buckets (two passes); range
    buckets above 256 are unsupported; histogram, radix digits and batched
    stay at 256."""
    from paper_1701_01189_amd.binding import BucketFnC
    ki, ko, ws = fake(0x1000000), fake(0x9000000), fake(0x20000000)
    n = 1000
    need = L.ms_workspace_size(0, n, 4096, 0, None)
    assert need >= 4 * n
    assert L.ms_workspace_size(1, n, 4096, 0, None) >= 8 * n
    assert L.ms_workspace_size(0, n, 65537, 0, None) == 0
    fn = BucketFnC(0, 20, 4095, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 65537, ctypes.byref(fn), ws, need, None, None) == -1
    assert L.ms_keys(ki, ko, None, n, 4096, ctypes.byref(fn), ws, need - 1, None, None) == -2
    bad = BucketFnC(0, 20, 8191, 0, None, None)
    assert L.ms_keys(ki, ko, None, n, 4096, ctypes.byref(bad), ws, need, None, None) == -4
    spl = BucketFnC(2, 0, 0, 0, fake(0x30000000), None)
    assert L.ms_keys(ki, ko, None, n, 1000, ctypes.byref(spl), ws, 1 << 30, None, None) == -6
    assert L.ms_histogram(ki, n, 1000, ctypes.byref(fn), fake(0x40000000), ws, need, None,
                          None) == -1


def test_sssp_host_checks(L):
    from paper_1701_01189_amd.binding import SsspStatsC
    sz = L.ms_sssp_workspace_size
    assert sz(1000, 5000, 10) > 0
    assert sz(0, 5, 10) == 0 and sz(5, 5, 1) == 0 and sz(5, 5, 257) == 0
    assert sz(1 << 31, 1 << 31, 10) == 0  # nv + ne must stay below 2^32 - 1
    row, col, wt, dist = fake(0x1000000), fake(0x2000000), fake(0x3000000), fake(0x4000000)
    ws = fake(0x20000000)
    need = sz(100, 400, 10)
    st = SsspStatsC()

    def call(nv=100, ne=400, src=0, delta=50, nb=10, r=row, c=col, w=wt, d=dist, wsb=need):
        return L.ms_sssp(r, c, w, nv, ne, src, delta, nb, d, ws, wsb, ctypes.byref(st), None)

    invalid, workspace = -1, -2
    assert call(nv=0) == invalid
    assert call(src=100) == invalid
    assert call(delta=0) == invalid
    assert call(nb=1) == invalid and call(nb=257) == invalid
    assert call(r=None) == invalid and call(d=None) == invalid
    assert call(c=None) == invalid and call(w=None) == invalid
    assert call(nv=1 << 31, ne=1 << 31) == invalid
    assert call(wsb=need - 1) == workspace


def test_plan_near_2e32_keeps_chunk_lengths_in_range(L):
    from paper_1701_01189_amd.binding import OptionsC
    n = (1 << 32) - 2  # the largest accepted size
    one = OptionsC()
    one.max_chunks = 1  # asks for a single chunk, whose length would not fit 32 bits
    assert L.ms_workspace_size(1, n, 32, 0, ctypes.byref(one)) > 0
    assert L.ms_workspace_size(1, n, 32, 0, None) > 0
    assert L.ms_workspace_size(1, n + 1, 32, 0, None) == 0
