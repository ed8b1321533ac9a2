"""Pins the CPU oracle to things other than itself (runs without a GPU).

* Eq. (1) of Section 4.2 evaluated by brute force on tiny inputs, in plain
  Python, compared with the oracle's counting-sort multisplit.
* Library routines: numpy's stable argsort (stable multisplit = stable sort
  by bucket id), numpy's searchsorted (upper bound over splitters), numpy's
  sort (radix sort result), Python integer division (delta buckets).
* Invariants of a stable multisplit, special cases (m = 1, one bucket, m = 2
  as a two-way split), the worked example of the localization figure and
  the LSD identity of Section 7.1.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_force_positions(b):
    """Eq. (1): p(i) = #{r : b_r < b_i} + #{r < i : b_r = b_i}."""
    n = len(b)
    p = []
    for i in range(n):
        glob = sum(1 for r in range(n) if b[r] < b[i])
        loc = sum(1 for r in range(i) if b[r] == b[i])
        p.append(glob + loc)
    return p


def py_bucket(k, kind, m, shift=0, mask=0, divisor=0, spl=None):
    if kind == oracle.SHIFT_MASK:
        return (k >> shift) & mask
    if kind == oracle.DIV:
        return k // divisor
    return sum(1 for s in spl if s <= k)


def kind_params(kind, m, seed):
    if kind == oracle.SHIFT_MASK:
        r = max(1, (m - 1).bit_length())
        return dict(shift=32 - r if m > 1 else 0, mask=m - 1)
    if kind == oracle.DIV:
        return dict(divisor=min(-(-(1 << 32) // m), 0xFFFFFFFF))
    spl = np.sort(inputs.uniform_u32(seed + 99, m - 1))
    return dict(splitters=spl)


MS = [1, 2, 3, 5, 8, 31, 32, 33, 64, 100, 255, 256]


@pytest.mark.parametrize("m", MS)
@pytest.mark.parametrize("kind", [oracle.SHIFT_MASK, oracle.DIV, oracle.SPLITTERS])
def test_eq1_brute_force(m, kind):
    for n in (0, 1, 2, 17, 64, 131):
        seed = 1000 * m + n + 7 * kind
        keys = inputs.uniform_u32(seed, n)
        vals = inputs.index_values(n)
        kp = kind_params(kind, m, seed)
        if kind == oracle.SHIFT_MASK and m & (m - 1):
            continue  # shift/mask needs power-of-two m to stay in range
        ok, ov, off = oracle.multisplit(keys, m, kind, vals=vals, **kp)
        b = [py_bucket(int(k), kind, m, spl=kp.get("splitters"),
                       shift=kp.get("shift", 0), mask=kp.get("mask", 0),
                       divisor=kp.get("divisor", 0)) for k in keys]
        p = brute_force_positions(b)
        for i in range(n):
            assert ok[p[i]] == keys[i]
            assert ov[p[i]] == vals[i]
        for j in range(m + 1):
            assert off[j] == sum(1 for x in b if x < j)


@pytest.mark.parametrize("m,kind", [(8, oracle.SHIFT_MASK), (32, oracle.SHIFT_MASK),
                                    (256, oracle.SHIFT_MASK), (7, oracle.DIV),
                                    (100, oracle.DIV), (256, oracle.SPLITTERS),
                                    (13, oracle.SPLITTERS)])
def test_matches_stable_argsort(m, kind):
    n = 200_003
    keys = inputs.uniform_u32(5 + m, n)
    vals = inputs.index_values(n)
    kp = kind_params(kind, m, 11)
    ok, ov, off = oracle.multisplit(keys, m, kind, vals=vals, **kp)
    if kind == oracle.SHIFT_MASK:
        b = (keys >> np.uint32(kp["shift"])) & np.uint32(kp["mask"])
    elif kind == oracle.DIV:
        b = keys.astype(np.int64) // kp["divisor"]
    else:
        b = np.searchsorted(kp["splitters"], keys, side="right")
    order = np.argsort(b, kind="stable")
    np.testing.assert_array_equal(ok, keys[order])
    np.testing.assert_array_equal(ov, vals[order])
    cnt = np.bincount(b, minlength=m)
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(cnt)]))


def test_bucket_ids_against_library():
    keys = np.concatenate([inputs.uniform_u32(3, 50_000),
                           np.array([0, 1, 2**31, 2**32 - 2, 2**32 - 1], dtype=np.uint32)])
    for m in (2, 3, 7, 100, 255, 256):
        d = -(-(1 << 32) // m)
        got = oracle.bucket_ids(keys, m, oracle.DIV, divisor=d)
        np.testing.assert_array_equal(got, np.array([int(k) // d for k in keys], dtype=np.uint32))
    spl = np.sort(inputs.uniform_u32(4, 255))
    spl[10:20] = spl[10]  # duplicate splitters give zero-width buckets
    spl = np.sort(spl)
    keys2 = np.concatenate([keys, spl, spl - np.uint32(1), spl + np.uint32(1)])
    got = oracle.bucket_ids(keys2, 256, oracle.SPLITTERS, splitters=spl)
    np.testing.assert_array_equal(got, np.searchsorted(spl, keys2, side="right"))
    got = oracle.bucket_ids(keys, 256, oracle.SHIFT_MASK, shift=8, mask=255)
    np.testing.assert_array_equal(got, (keys >> np.uint32(8)) & np.uint32(255))


def check_invariants(keys, vals, ok, ov, off, b_of, m):
    n = len(keys)
    # permutation: same multiset of keys; values (original index) a permutation
    np.testing.assert_array_equal(np.sort(ok), np.sort(keys))
    np.testing.assert_array_equal(np.sort(ov), np.arange(n, dtype=np.uint32))
    bo = b_of(ok)
    assert np.all(np.diff(bo.astype(np.int64)) >= 0)  # buckets ascending
    cnt = np.bincount(b_of(keys), minlength=m)
    np.testing.assert_array_equal(off[1:] - off[:-1], cnt)
    assert off[0] == 0 and off[m] == n
    for j in range(m):
        seg = ov[off[j]:off[j + 1]]
        assert np.all(bo[off[j]:off[j + 1]] == j)
        assert np.all(np.diff(seg.astype(np.int64)) > 0)  # stable
    np.testing.assert_array_equal(keys[ov], ok)


@pytest.mark.parametrize("m", [2, 8, 32, 256])
def test_invariants_uniform_and_skewed(m):
    n = 100_000
    vals = inputs.index_values(n)
    r = (m - 1).bit_length()
    for dist in ("uniform", "binomial", "alpha"):
        keys = inputs.skewed_bucket_keys(17, n, m, dist)
        ok, ov, off = oracle.multisplit(keys, m, oracle.SHIFT_MASK, vals=vals, shift=32 - r,
                                        mask=m - 1)
        check_invariants(keys, vals, ok, ov, off,
                         lambda a: (a >> np.uint32(32 - r)) & np.uint32(m - 1), m)
        ko, _, off2 = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=32 - r, mask=m - 1)
        np.testing.assert_array_equal(ko, ok)  # key-only = keys of key-value
        np.testing.assert_array_equal(off2, off)


def test_special_cases():
    n = 5000
    keys = inputs.uniform_u32(21, n)
    vals = inputs.index_values(n)
    # m = 1: identity permutation
    ok, ov, off = oracle.multisplit(keys, 1, oracle.SHIFT_MASK, vals=vals, shift=0, mask=0)
    np.testing.assert_array_equal(ok, keys)
    np.testing.assert_array_equal(off, [0, n])
    # every key in one bucket: identity
    ok, ov, off = oracle.multisplit(keys | np.uint32(0xE0000000), 8, oracle.SHIFT_MASK,
                                    vals=vals, shift=29, mask=7)
    np.testing.assert_array_equal(ov, vals)
    assert list(off) == [0] * 8 + [n]
    # m = 2: a two-way stable split (Section 3.2)
    ok, ov, off = oracle.multisplit(keys, 2, oracle.SHIFT_MASK, vals=vals, shift=31, mask=1)
    lo = [int(k) for k in keys if k < 2**31]
    hi = [int(k) for k in keys if k >= 2**31]
    assert list(map(int, ok)) == lo + hi
    # empty input
    ok, ov, off = oracle.multisplit(keys[:0], 16, oracle.SHIFT_MASK, vals=vals[:0], shift=28,
                                    mask=15)
    assert len(ok) == 0 and list(off) == [0] * 17


def test_worked_example_localization_figure():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "localization_example.txt"))
            if l.strip() and not l.startswith("#")]
    in_j = [int(r[1]) for r in rows]
    want = [int(r[2]) for r in rows]
    # bucket j = 1; the other elements go to buckets 0 and 2 alternately
    b = []
    other = 0
    for x in in_j:
        if x:
            b.append(1)
        else:
            b.append(0 if other % 2 == 0 else 2)
            other += 1
    keys = np.array([(bb << 30) | i for i, bb in enumerate(b)], dtype=np.uint32)
    vals = np.arange(len(keys), dtype=np.uint32)
    ok, ov, off = oracle.multisplit(keys, 4, oracle.SHIFT_MASK, vals=vals, shift=30, mask=3)
    pos = np.empty(len(keys), dtype=np.int64)
    pos[ov] = np.arange(len(keys))
    for i in range(len(keys)):
        if in_j[i]:
            assert pos[i] - off[1] == want[i]
    assert off[2] - off[1] == 6


def test_radix_sort_against_library_and_lsd_identity():
    n = 300_000
    keys = inputs.uniform_u32(105, n)
    keys[::7] = keys[3]  # many equal keys so stability is observable
    vals = inputs.index_values(n)
    ok, ov = oracle.radix_sort(keys, vals)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(ok, keys[order])
    np.testing.assert_array_equal(ov, vals[order])
    # Section 7.1: 4 stable multisplits on 8-bit digits, least significant first
    k, v = keys, vals
    for p in range(4):
        k, v, _ = oracle.multisplit(k, 256, oracle.SHIFT_MASK, vals=v, shift=8 * p, mask=255)
    np.testing.assert_array_equal(k, ok)
    np.testing.assert_array_equal(v, ov)


def test_batched_equals_per_instance():
    sizes = inputs.batched_sizes(104, 40, 2, 12)
    seg = inputs.segment_offsets(sizes)
    keys, vals = inputs.batched_pairs(104, sizes)
    ok, ov, off = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    for i in range(len(sizes)):
        a, z = int(seg[i]), int(seg[i + 1])
        k1, v1, o1 = oracle.multisplit(keys[a:z], 64, oracle.SHIFT_MASK, vals=vals[a:z],
                                       shift=8, mask=63)
        np.testing.assert_array_equal(ok[a:z], k1)
        np.testing.assert_array_equal(ov[a:z], v1)
        np.testing.assert_array_equal(off[i * 65:(i + 1) * 65], o1)
        assert off[i * 65 + 64] == z - a


def test_brute_force_detects_planted_mistake():
    """The Eq. (1) check fails on an oracle output with two entries swapped."""
    keys = inputs.uniform_u32(77, 40)
    vals = inputs.index_values(40)
    ok, ov, off = oracle.multisplit(keys, 4, oracle.SHIFT_MASK, vals=vals, shift=30, mask=3)
    b = [int(k) >> 30 for k in keys]
    p = brute_force_positions(b)
    ov = ov.copy()
    j = int(off[1])  # swap two entries of one bucket: breaks stability only
    ov[j], ov[j + 1] = ov[j + 1], ov[j]
    assert any(ov[p[i]] != vals[i] for i in range(40))


@pytest.mark.parametrize("m", [257, 1000, 4096, 65536])
def test_oracle_more_than_256_buckets_matches_stable_argsort(m):
    """The oracle's counting sort has no bucket limit: pinned by numpy's
    stable argsort of the bucket ids (shift/mask and delta buckets)."""
    n = 20_011
    keys = inputs.uniform_u32(m, n)
    vals = inputs.index_values(n)
    r = (m - 1).bit_length()
    d = -(-(1 << 32) // m)
    for kind, kw, ids in ((oracle.SHIFT_MASK, dict(shift=32 - r, mask=(1 << r) - 1),
                           keys >> np.uint32(32 - r)),
                          (oracle.DIV, dict(divisor=d), (keys.astype(np.uint64) // d))):
        mm = 1 << r if kind == oracle.SHIFT_MASK else m
        k, v, off = oracle.multisplit(keys, mm, kind, vals=vals, **kw)
        order = np.argsort(ids, kind="stable")
        np.testing.assert_array_equal(v, vals[order])
        np.testing.assert_array_equal(k, keys[order])
        np.testing.assert_array_equal(np.diff(off.astype(np.int64)),
                                      np.bincount(ids.astype(np.int64), minlength=mm))
