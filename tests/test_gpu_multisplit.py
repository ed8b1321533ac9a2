"""GPU parity: the gfx950 multisplit against the CPU oracle, element by element.

Every comparison is bit-exact (integer work).  Small cases span several tiles
and ragged tails for every reordering mode and workgroup shape; the workload
sizes are compared in full against the oracle where it finishes in seconds,
and through properties that pin the unique stable result otherwise (a stable
multisplit is the only permutation with ascending buckets and increasing
original indices inside every bucket).
"""
import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def say(*a):
    print(*a, flush=True)


SHAPES = [  # (reorder, waves_per_block, items_per_lane)
    (1, 8, 8), (1, 8, 4), (1, 4, 8), (1, 4, 16), (1, 16, 8), (2, 8, 8), (2, 4, 16), (3, 8, 8)]


def fn_for(kind, m, seed=0):
    """(gpu BucketFn, oracle kwargs, oracle kind, splitter array or None)."""
    from paper_1701_01189_amd import binding as ms
    if kind == "shift":
        r = (m - 1).bit_length()
        shift = 32 - r if r > 0 else 0
        return ms.BucketFn.shift_mask(shift, m - 1), dict(shift=shift, mask=m - 1), \
            oracle.SHIFT_MASK, None
    if kind == "div":
        d = -(-(1 << 32) // m)
        if d > 0xFFFFFFFF:
            d = 0xFFFFFFFF
        return ms.BucketFn.div(d), dict(divisor=d), oracle.DIV, None
    spl = np.sort(inputs.uniform_u32(seed + 5, m - 1)) if m > 1 else np.zeros(1, np.uint32)
    t = dev(spl)
    return ms.BucketFn.splitter(t), dict(splitters=spl[:m - 1]), oracle.SPLITTERS, t


def check_case(n, m, kind, kv, shape, seed, prescan=0):
    from paper_1701_01189_amd import binding as ms
    if kind == "shift" and m & (m - 1):
        return
    if kind == "div" and m == 1:
        return
    keys = inputs.uniform_u32(seed, n)
    vals = inputs.index_values(n)
    fn, okw, okind, _keep = fn_for(kind, m, seed)
    ek, ev, eo = oracle.multisplit(keys, m, okind, vals=vals if kv else None, **okw)
    opt = ms.Options(reorder=shape[0], waves_per_block=shape[1], items_per_lane=shape[2],
                     prescan=prescan)
    say("case n=%d m=%d kind=%s kv=%d shape=%s seed=%d prescan=%d" % (n, m, kind, kv, shape,
                                                                      seed, prescan))
    if kv:
        k, v, o = ms.pairs(dev(keys), dev(vals), m, fn, options=opt)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(v), ev)
    else:
        k, o = ms.keys(dev(keys), m, fn, options=opt)
        torch.cuda.synchronize()
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("shape", SHAPES)
def test_small_shapes_ragged(shape):
    combos = [(1, 1), (63, 2), (64, 8), (65, 3), (4095, 32), (4097, 33), (8193, 64),
              (12345, 65), (30001, 128), (100003, 200), (70001, 256), (5000, 255)]
    for i, (n, m) in enumerate(combos):
        for kind in ("shift", "div", "splitters"):
            check_case(n, m, kind, kv=(i % 2 == 0), shape=shape, seed=11 * i + 3)


@pytest.mark.parametrize("prescan", [1, 2])  # ballot histogram, lane counters
def test_prescan_methods(prescan):
    """Both pre-scan histograms under block reordering, every bucket kind."""
    combos = [(1, 1), (65, 3), (4097, 33), (30001, 128), (100003, 200), (262147, 256),
              (524309, 32), (70001, 64)]
    for i, (n, m) in enumerate(combos):
        for kind in ("shift", "div", "splitters"):
            for shape in ((1, 8, 8), (1, 4, 8), (1, 4, 16), (1, 16, 8)):
                check_case(n, m, kind, kv=(i % 2 == 1), shape=shape, seed=5 * i + 1,
                           prescan=prescan)


@pytest.mark.parametrize("prescan", [1, 2])
def test_prescan_methods_one_bucket(prescan):
    """Every key in one bucket (the worst case for same-address LDS traffic)."""
    from paper_1701_01189_amd import binding as ms
    n = 200_003
    keys = inputs.uniform_u32(19, n) & np.uint32(0x00FFFFFF) | np.uint32(0x7B000000)
    for m, shift in ((256, 24), (32, 27), (2, 31)):
        ek, _, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=shift, mask=m - 1)
        say("case one-bucket prescan=%d m=%d" % (prescan, m))
        k, o = ms.keys(dev(keys), m, ms.BucketFn.shift_mask(shift, m - 1),
                       options=ms.Options(reorder=1, prescan=prescan))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("m", [2, 8, 32, 256])
def test_several_chunks_per_group(shape, m):
    # small max_chunks forces many tiles per chunk: running bases carry over tiles
    from paper_1701_01189_amd import binding as ms
    n = 300_007
    keys = inputs.uniform_u32(77 + m, n)
    vals = inputs.index_values(n)
    r = (m - 1).bit_length()
    ek, ev, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals, shift=32 - r, mask=m - 1)
    for chunks in (1, 3, 7):
        say("case chunks=%d m=%d shape=%s" % (chunks, m, shape))
        opt = ms.Options(reorder=shape[0], waves_per_block=shape[1], items_per_lane=shape[2],
                         max_chunks=chunks)
        k, v, o = ms.pairs(dev(keys), dev(vals), m, ms.BucketFn.shift_mask(32 - r, m - 1),
                           options=opt)
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("m", [2, 32, 256])
def test_several_chunks_per_group_keys(shape, m):
    # Key-only tiles with many tiles per chunk: the running bucket bases are
    # carried over the chunk's tiles (visited last to first by block and wave
    # reordering) without values in the tile.
    from paper_1701_01189_amd import binding as ms
    n = 300_007
    keys = inputs.uniform_u32(91 + m, n)
    r = (m - 1).bit_length()
    ek, _, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=32 - r, mask=m - 1)
    for chunks in (1, 3, 7):
        say("case keys chunks=%d m=%d shape=%s" % (chunks, m, shape))
        opt = ms.Options(reorder=shape[0], waves_per_block=shape[1], items_per_lane=shape[2],
                         max_chunks=chunks)
        k, o = ms.keys(dev(keys), m, ms.BucketFn.shift_mask(32 - r, m - 1), options=opt)
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)


def test_empty_and_single_bucket():
    from paper_1701_01189_amd import binding as ms
    say("case n=0")
    k, o = ms.keys(dev(np.zeros(0, np.uint32)), 16, ms.BucketFn.shift_mask(28, 15))
    assert host(o).tolist() == [0] * 17
    n = 50_000
    keys = inputs.uniform_u32(9, n) | np.uint32(0xF0000000)
    vals = inputs.index_values(n)
    for shape in SHAPES:
        say("case one-bucket shape=%s" % (shape,))
        opt = ms.Options(*shape)
        k, v, o = ms.pairs(dev(keys), dev(vals), 16, ms.BucketFn.shift_mask(28, 15), options=opt)
        np.testing.assert_array_equal(host(k), keys)
        np.testing.assert_array_equal(host(v), vals)
        assert host(o).tolist() == [0] * 15 + [0, n]


@pytest.mark.parametrize("dist", ["binomial", "alpha"])
def test_skewed_m256(dist):
    from paper_1701_01189_amd import binding as ms
    n = 1 << 22
    keys = inputs.skewed_bucket_keys(100, n, 256, dist)
    vals = inputs.index_values(n)
    ek, ev, eo = oracle.multisplit(keys, 256, oracle.SHIFT_MASK, vals=vals, shift=24, mask=255)
    for shape in SHAPES:
        say("case skew=%s shape=%s" % (dist, shape))
        k, v, o = ms.pairs(dev(keys), dev(vals), 256, ms.BucketFn.shift_mask(24, 255),
                           options=ms.Options(*shape))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)


def test_keys_2e20_m8():
    """Key-only multisplit, n = 2^20 uniform keys (seed 101), m = 8, f = k >> 29."""
    from paper_1701_01189_amd import binding as ms
    n = 1 << 20
    keys = inputs.uniform_u32(101, n)
    ek, _, eo = oracle.multisplit(keys, 8, oracle.SHIFT_MASK, shift=29, mask=7)
    for shape in SHAPES:
        say("case keys 2^20 m=8 shape=%s" % (shape,))
        k, o = ms.keys(dev(keys), 8, ms.BucketFn.shift_mask(29, 7), options=ms.Options(*shape))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)
        assert len(host(o)) == 9


def test_pairs_2e25_m32_reorder_sweep():
    """Key-value multisplit, n = 2^25 (seed 102), values = index, m = 32, f = k >> 27."""
    from paper_1701_01189_amd import binding as ms
    n = 1 << 25
    keys = inputs.uniform_u32(102, n)
    vals = inputs.index_values(n)
    ek, ev, eo = oracle.multisplit(keys, 32, oracle.SHIFT_MASK, vals=vals, shift=27, mask=31)
    dk, dv = dev(keys), dev(vals)
    for shape in SHAPES + [(0, 0, 0)]:
        say("case pairs 2^25 m=32 shape=%s" % (shape,))
        k, v, o = ms.pairs(dk, dv, 32, ms.BucketFn.shift_mask(27, 31), options=ms.Options(*shape))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)


def test_repeated_calls_deterministic():
    from paper_1701_01189_amd import binding as ms
    n = 1 << 21
    keys = inputs.uniform_u32(5, n)
    vals = inputs.index_values(n)
    dk, dv = dev(keys), dev(vals)
    ref = None
    for rep in range(5):
        say("case repeat %d" % rep)
        k, v, o = ms.pairs(dk, dv, 64, ms.BucketFn.shift_mask(26, 63))
        cur = (host(k), host(v), host(o))
        if ref is None:
            ref = cur
            ek, ev, eo = oracle.multisplit(keys, 64, oracle.SHIFT_MASK, vals=vals, shift=26,
                                           mask=63)
            np.testing.assert_array_equal(cur[0], ek)
        for a, b in zip(ref, cur):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5, 6, 7, 8])
def test_identity_buckets_sort_small_keys(bits):
    """Identity buckets over keys of `bits` bits (f(k) = k, m = 2^bits): the
    multisplit is then the stable sort of those keys (Section 7.1's sweep)."""
    from paper_1701_01189_amd import binding as ms
    m = 1 << bits
    n = (1 << 20) + 7
    keys = inputs.uniform_u32(120 + bits, n) & np.uint32(m - 1)
    vals = inputs.index_values(n)
    order = np.argsort(keys, kind="stable")
    ek, ev, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals, shift=0, mask=m - 1)
    np.testing.assert_array_equal(ev, vals[order])  # pin of the oracle itself
    for shape in [(0, 0, 0), (2, 8, 8), (3, 8, 8)]:
        say("case identity bits=%d shape=%s" % (bits, shape))
        k, v, o = ms.pairs(dev(keys), dev(vals), m, ms.BucketFn.shift_mask(0, m - 1),
                           options=ms.Options(*shape))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("m,kv", [(8, False), (32, False), (32, True), (128, True)])
def test_whole_line_stores(m, kv):
    """From 2^22 elements on, the elements of whole 128-byte output lines are
    stored nontemporally (up to 64 buckets; key-value tiles above).  Ragged n,
    several tile shapes, and outputs that start 4 bytes past a line boundary,
    where the whole-line test no longer matches the real lines: still exact."""
    from paper_1701_01189_amd import binding as ms
    n = (1 << 22) + 777
    keys = inputs.uniform_u32(120 + m, n)
    vals = inputs.index_values(n)
    shift = 32 - (m - 1).bit_length()
    ek, ev, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals if kv else None,
                                   shift=shift, mask=m - 1)
    dk, dv = dev(keys), dev(vals)
    fn = ms.BucketFn.shift_mask(shift, m - 1)
    for off in (0, 1):
        for shape in [(1, 8, 8), (1, 4, 16), (1, 16, 8), (0, 0, 0)]:
            say("case whole lines m=%d kv=%d offset=%d shape=%s" % (m, kv, off, shape))
            kbuf = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
            vbuf = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
            ko, vo = kbuf[off:off + n], vbuf[off:off + n]
            if kv:
                ms.pairs(dk, dv, m, fn, keys_out=ko, vals_out=vo, options=ms.Options(*shape))
                np.testing.assert_array_equal(host(vo), ev)
                k, o = ko, None
            else:
                k, o = ms.keys(dk, m, fn, keys_out=ko, options=ms.Options(*shape))
                np.testing.assert_array_equal(host(o), eo)
            np.testing.assert_array_equal(host(k), ek)
            # nothing outside the output
            assert int(kbuf[n if off == 0 else 0].item()) == 0
