"""GPU parity of the multisplit LSD radix sort (Section 7.1) against the
oracle's stable sort, and at full size through properties that determine the
stable sort uniquely (sorted keys; values = original index form a
permutation that reproduces the keys; increasing indices among equal keys)."""
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


@pytest.mark.parametrize("bits", [8, 7, 4, 1])
@pytest.mark.parametrize("kv", [True, False])
def test_radix_sort_vs_oracle(bits, kv):
    from paper_1701_01189_amd import binding as ms
    n = 100_003 if bits >= 4 else 5_003
    keys = inputs.uniform_u32(105, n)
    keys[::5] = keys[7]  # ties make stability observable
    vals = inputs.index_values(n)
    ek, ev = oracle.radix_sort(keys, vals)
    print("case radix n=%d bits=%d kv=%d" % (n, bits, kv), flush=True)
    k, v = ms.radix_sort(dev(keys), dev(vals) if kv else None, bits_per_pass=bits)
    np.testing.assert_array_equal(host(k), ek)
    if kv:
        np.testing.assert_array_equal(host(v), ev)


def test_radix_sort_2e28_pairs_properties():
    """n = 2^28 uniform keys (seed 105), values = index, 4 passes of 8 bits."""
    from paper_1701_01189_amd import binding as ms
    n = 1 << 28
    keys = inputs.uniform_u32(105, n)
    vals = inputs.index_values(n)
    print("case radix 2^28 pairs", flush=True)
    k, v = ms.radix_sort(dev(keys), dev(vals), bits_per_pass=8)
    torch.cuda.synchronize()
    hk, hv = host(k), host(v)
    del k, v
    assert np.all(hk[1:] >= hk[:-1])
    np.testing.assert_array_equal(keys[hv], hk)   # a permutation carrying its keys
    eq = hk[1:] == hk[:-1]
    assert np.all(hv[1:][eq] > hv[:-1][eq])       # stable
    # sampled ranks: position = number of smaller keys + earlier equal keys
    rng = np.random.default_rng(0)
    for p in rng.integers(0, n, 4):
        key, idx = hk[p], int(hv[p])
        smaller = int(np.count_nonzero(keys < key))
        earlier_equal = int(np.count_nonzero(keys[:idx] == key))
        assert p == smaller + earlier_equal
