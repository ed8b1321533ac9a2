"""GPU multisplit past 2^31 elements, where any index held in a signed 32-bit
integer would overflow, up to the largest size the library takes (2^32 - 2).

At this size the oracle is too slow to run element by element, so the output
is checked against the properties that determine the unique stable
multisplit, all computed on the GPU in slices:
  * output bucket ids never decrease;
  * per-bucket counts equal the input's, and the bucket starts are their
    exclusive prefix sum (offsets[m] = n);
  * with values = original index: each output value, used to gather the
    input key, gives the output key (the value names an input element of
    that bucket), and values strictly increase inside every bucket (input
    order kept).  With the counts, these make the output the stable
    multisplit.
Inputs: uniform keys from a seeded torch generator on the GPU.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SLICE = 1 << 28


def say(*a):
    print(*a, flush=True)


def u32(t):
    """int32 tensor holding uint32 values -> int64 values."""
    return t.to(torch.int64) & 0xFFFFFFFF


def buckets(keys_i32, kind, m, param):
    k = u32(keys_i32)
    if kind == "shift":
        return (k >> param) & (m - 1)
    return k // param


def check_stable_multisplit(kin, ko, vo, off, n, m, kind, param):
    dev = kin.device
    cnt_in = torch.zeros(m, dtype=torch.int64, device=dev)
    cnt_out = torch.zeros(m, dtype=torch.int64, device=dev)
    prev_b, prev_v = None, None
    for s in range(0, n, SLICE):
        e = min(n, s + SLICE)
        cnt_in += torch.bincount(buckets(kin[s:e], kind, m, param), minlength=m)
        b = buckets(ko[s:e], kind, m, param)
        cnt_out += torch.bincount(b, minlength=m)
        assert bool((b[1:] >= b[:-1]).all()), "bucket ids decrease inside slice %d" % s
        if prev_b is not None:
            assert int(b[0]) >= prev_b
        if vo is not None:
            v = u32(vo[s:e])
            assert bool((kin[v] == ko[s:e]).all()), "value does not name its key (slice %d)" % s
            same = b[1:] == b[:-1]
            assert bool((v[1:][same] > v[:-1][same]).all()), "order not kept (slice %d)" % s
            if prev_b is not None and int(b[0]) == prev_b:
                assert int(v[0]) > prev_v
            prev_v = int(v[-1])
        prev_b = int(b[-1])
    assert bool((cnt_in == cnt_out).all())
    starts = torch.zeros(m + 1, dtype=torch.int64, device=dev)
    starts[1:] = torch.cumsum(cnt_out, 0)
    assert bool((u32(off) == starts).all())
    assert int(starts[-1]) == n


def test_pairs_past_2e31_shift_mask():
    from paper_1701_01189_amd import binding as ms
    n = (1 << 31) + 12345
    say("case large pairs n=%d m=32 shift" % n)
    g = torch.Generator(device="cuda").manual_seed(2031)
    kin = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda",
                        generator=g)
    vin = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in range(0, n, SLICE):  # values = index, wrapped into int32 storage
        e = min(n, s + SLICE)
        vin[s:e] = torch.arange(s, e, dtype=torch.int64, device="cuda").to(torch.int32)
    ko, vo, off = ms.pairs(kin, vin, 32, ms.BucketFn.shift_mask(27, 31))
    torch.cuda.synchronize()
    del vin
    check_stable_multisplit(kin, ko, vo, off, n, 32, "shift", 27)


def test_keys_past_2e31_delta_256():
    from paper_1701_01189_amd import binding as ms
    n = (1 << 31) + 777
    m, d = 256, 1 << 24
    say("case large keys n=%d m=%d delta" % (n, m))
    g = torch.Generator(device="cuda").manual_seed(2032)
    kin = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda",
                        generator=g)
    fn = ms.BucketFn.div(d)
    ko, off = ms.keys(kin, m, fn)
    torch.cuda.synchronize()
    check_stable_multisplit(kin, ko, None, off, n, m, "div", d)
    # The key-only output must equal the keys of the key-value output on the
    # same keys with values = original index.  The key-value output is pinned
    # to the unique stable multisplit by check_stable_multisplit (each value
    # names its input key, values increase inside every bucket, counts
    # match), so this pins the key-only output's multiset and its order
    # inside every bucket too.
    vin = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in range(0, n, SLICE):
        e = min(n, s + SLICE)
        vin[s:e] = torch.arange(s, e, dtype=torch.int64, device="cuda").to(torch.int32)
    say("case large pairs (same keys) n=%d m=%d delta" % (n, m))
    ko2, vo2, off2 = ms.pairs(kin, vin, m, fn)
    torch.cuda.synchronize()
    del vin
    check_stable_multisplit(kin, ko2, vo2, off2, n, m, "div", d)
    assert bool((off == off2).all())
    for s in range(0, n, SLICE):
        assert bool((ko[s:s + SLICE] == ko2[s:s + SLICE]).all()), "key-only differs at slice %d" % s


def test_pairs_at_the_largest_size():
    from paper_1701_01189_amd import binding as ms
    n = (1 << 32) - 2  # the largest n the library accepts
    say("case large pairs n=%d m=8 shift" % n)
    g = torch.Generator(device="cuda").manual_seed(2033)
    kin = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda",
                        generator=g)
    vin = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in range(0, n, SLICE):
        e = min(n, s + SLICE)
        vin[s:e] = torch.arange(s, e, dtype=torch.int64, device="cuda").to(torch.int32)
    ko, vo, off = ms.pairs(kin, vin, 8, ms.BucketFn.shift_mask(29, 7))
    torch.cuda.synchronize()
    del vin
    check_stable_multisplit(kin, ko, vo, off, n, 8, "shift", 29)
