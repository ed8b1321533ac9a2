"""The no-allocation entry point (ms_pairs_noalloc) against ms_pairs and the
oracle: two calls in a row on one GPU, the second with a smaller input, so
that it reads the static scratch array the first call left behind.  Key-value
and key-only, shift/mask and range buckets; bit-exact.  Called through the
C ABI (ctypes)."""
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


def run_both(keys, vals, m, fn):
    """(noalloc result, ms_pairs result) on the same device inputs."""
    from paper_1701_01189_amd import binding as ms
    dk = dev(keys)
    dv = dev(vals) if vals is not None else None
    n = len(keys)
    ko = torch.empty(n, dtype=torch.int32, device="cuda")
    vo = torch.empty(n, dtype=torch.int32, device="cuda") if vals is not None else None
    off = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    ms.pairs_noalloc(dk, dv, m, fn, ko, vo, off)
    if vals is not None:
        rk, rv, ro = ms.pairs(dk, dv, m, fn)
    else:
        rk, ro = ms.keys(dk, m, fn)
        rv = None
    torch.cuda.synchronize()
    got = (host(ko), host(vo) if vo is not None else None, host(off))
    ref = (host(rk), host(rv) if rv is not None else None, host(ro))
    return got, ref


@pytest.mark.parametrize("kv", [True, False])
def test_noalloc_twice_shift_mask(kv):
    from paper_1701_01189_amd import binding as ms
    m = 32
    fn = ms.BucketFn.shift_mask(27, 31)
    for i, n in enumerate([3_000_017, 123_457]):  # the second call is smaller
        print("noalloc shift_mask kv=%s call %d n=%d" % (kv, i, n), flush=True)
        keys = inputs.uniform_u32(700 + i, n)
        vals = inputs.index_values(n) if kv else None
        got, ref = run_both(keys, vals, m, fn)
        ek, ev, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals, shift=27, mask=31)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[0], ek)
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[2], eo)
        if kv:
            assert np.array_equal(got[1], ref[1]) and np.array_equal(got[1], ev)


def test_noalloc_twice_range_buckets_m256():
    from paper_1701_01189_amd import binding as ms
    m = 256
    spl = np.sort(inputs.uniform_u32(711, m - 1))
    dspl = dev(spl)
    fn = ms.BucketFn.splitter(dspl)
    for i, n in enumerate([2_000_003, 50_001]):
        print("noalloc splitters call %d n=%d" % (i, n), flush=True)
        keys = inputs.uniform_u32(720 + i, n)
        vals = inputs.index_values(n)
        got, ref = run_both(keys, vals, m, fn)
        ek, ev, eo = oracle.multisplit(keys, m, oracle.SPLITTERS, vals=vals, splitters=spl)
        for g, r, e in zip(got, ref, (ek, ev, eo)):
            assert np.array_equal(g, r) and np.array_equal(g, e)


def test_noalloc_rejects_wide_and_empty_is_ok():
    from paper_1701_01189_amd import binding as ms
    keys = inputs.uniform_u32(730, 1000)
    dk = dev(keys)
    ko = torch.empty_like(dk)
    off = torch.empty(4097, dtype=torch.int32, device="cuda")
    with pytest.raises(ms.MultisplitError) as e:
        ms.pairs_noalloc(dk, None, 4096, ms.BucketFn.shift_mask(20, 4095), ko, None, off)
    assert "MS_ERR_WORKSPACE" in str(e.value)
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    off9 = torch.full((9,), 7, dtype=torch.int32, device="cuda")
    ms.pairs_noalloc(empty, None, 8, ms.BucketFn.shift_mask(29, 7), empty, None, off9)
    torch.cuda.synchronize()
    assert np.array_equal(host(off9), np.zeros(9, np.uint32))
