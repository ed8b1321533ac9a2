"""GPU parity at the size the key-only roofline sweep is measured on:
n = 2^28 uniform keys (seed 100), delta buckets f(k) = k >> (32 - log2 m) as
shift/mask buckets, default tuning (the launch configuration the benchmark
times), compared element by element with the CPU oracle, keys and bucket
starts, at m = 2, 32 and 256; and the same keys as key-value pairs at m = 32.
"""
import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 1 << 28


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def keys():
    return inputs.uniform_u32(100, N)


def _host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("m", [2, 32, 256])
def test_keys_2e28_default_tuning(keys, m):
    from paper_1701_01189_amd import binding as ms
    r = (m - 1).bit_length()
    say("case keys n=2^28 m=%d shift=%d default tuning" % (m, 32 - r))
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    k, o = ms.keys(dk, m, ms.BucketFn.shift_mask(32 - r, m - 1))
    torch.cuda.synchronize()
    del dk
    ek, _, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=32 - r, mask=m - 1)
    np.testing.assert_array_equal(_host(o), eo)
    got = _host(k)
    del k
    np.testing.assert_array_equal(got, ek)


def test_pairs_2e28_m32_default_tuning(keys):
    from paper_1701_01189_amd import binding as ms
    say("case pairs n=2^28 m=32 default tuning")
    vals = inputs.index_values(N)
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    dv = torch.from_numpy(vals.view(np.int32)).cuda()
    k, v, o = ms.pairs(dk, dv, 32, ms.BucketFn.shift_mask(27, 31))
    torch.cuda.synchronize()
    del dk, dv
    ek, ev, eo = oracle.multisplit(keys, 32, oracle.SHIFT_MASK, vals=vals, shift=27, mask=31)
    np.testing.assert_array_equal(_host(o), eo)
    np.testing.assert_array_equal(_host(k), ek)
    np.testing.assert_array_equal(_host(v), ev)
