"""GPU parity of multisplit into more than 256 buckets (up to 65536;
shift/mask and delta buckets, two stable byte-digit passes) against the
oracle, bit-exact: keys, values and all m + 1 bucket starts."""
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


def fns(m):
    from paper_1701_01189_amd import binding as ms
    out = []
    r = (m - 1).bit_length()
    if m & (m - 1) == 0:
        out.append(("shift", ms.BucketFn.shift_mask(32 - r, m - 1), oracle.SHIFT_MASK,
                    dict(shift=32 - r, mask=m - 1)))
    # low bits as the bucket (identity-like; the second pass sees small shifts)
    out.append(("lowmask", ms.BucketFn.shift_mask(3, (1 << (r - 1)) - 1), oracle.SHIFT_MASK,
                dict(shift=3, mask=(1 << (r - 1)) - 1)))
    d = min(-(-(1 << 32) // m), 0xFFFFFFFF)
    out.append(("div", ms.BucketFn.div(d), oracle.DIV, dict(divisor=d)))
    return out


@pytest.mark.parametrize("m", [257, 300, 1000, 4096, 65536])
def test_wide_vs_oracle(m):
    from paper_1701_01189_amd import binding as ms
    for i, n in enumerate([0, 1, 1000, 100_003, (1 << 20) + 3]):
        keys = inputs.uniform_u32(500 + m + i, n)
        vals = inputs.index_values(n)
        for name, fn, kind, kw in fns(m):
            say("case wide m=%d n=%d %s" % (m, n, name))
            ek, ev, eo = oracle.multisplit(keys, m, kind, vals=vals, **kw)
            k, v, o = ms.pairs(dev(keys), dev(vals), m, fn)
            np.testing.assert_array_equal(host(o), eo)
            np.testing.assert_array_equal(host(k), ek)
            np.testing.assert_array_equal(host(v), ev)
            if n == 100_003:
                k2, o2 = ms.keys(dev(keys), m, fn, options=ms.Options(reorder=2))
                np.testing.assert_array_equal(host(k2), ek)
                np.testing.assert_array_equal(host(o2), eo)


def test_wide_skew_and_full_size():
    """All keys in two far-apart buckets (long runs of empty buckets between
    the starts), and 2^25 pairs at m = 4096 in full."""
    from paper_1701_01189_amd import binding as ms
    m = 65536
    n = 200_001
    keys = inputs.uniform_u32(77, n)
    keys = np.where(keys & np.uint32(1), np.uint32(0x0000FFFF), np.uint32(0xFFFF0000)).astype(np.uint32)
    ek, _, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=16, mask=m - 1)
    say("case wide two-bucket skew")
    k, o = ms.keys(dev(keys), m, ms.BucketFn.shift_mask(16, m - 1))
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)
    n = 1 << 25
    keys = inputs.uniform_u32(130, n)
    vals = inputs.index_values(n)
    ek, ev, eo = oracle.multisplit(keys, 4096, oracle.SHIFT_MASK, vals=vals, shift=20, mask=4095)
    say("case wide 2^25 pairs m=4096")
    k, v, o = ms.pairs(dev(keys), dev(vals), 4096, ms.BucketFn.shift_mask(20, 4095))
    np.testing.assert_array_equal(host(o), eo)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(v), ev)
