"""GPU checks of the autotuner (ms_autotune) and its JSON cache (tuning.py).

The autotuner times every candidate tuning on the caller's buffers and returns
the fastest one.  Which candidate wins depends on the machine, so the tests
check what holds for any winner: it is one of the candidates, fields that are
not tuned come from `base`, its time is positive, and the operation run with
the returned options gives the oracle's result bit for bit.
"""
import json

import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (reorder, waves per workgroup, windows per wavefront) tried for multisplits
# and radix sorts; (waves, windows, claim) tried for batched.
MULTI = {(1, 8, 8), (1, 8, 4), (1, 4, 8), (1, 4, 16), (1, 16, 8), (1, 16, 16), (2, 8, 8),
         (2, 4, 16), (3, 8, 8)}
BATCH = {(8, 8, 4), (8, 8, 16), (8, 8, 32), (8, 4, 4), (8, 4, 16), (8, 4, 32), (4, 16, 16),
         (4, 8, 16), (16, 4, 16), (16, 4, 32), (16, 8, 16), (16, 8, 32)}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("kv", [False, True])
@pytest.mark.parametrize("m", [2, 32, 256])
def test_autotune_multisplit_winner_matches_oracle(kv, m):
    from paper_1701_01189_amd import binding as ms
    n = (1 << 20) + 777
    keys = inputs.uniform_u32(300 + m, n)
    vals = inputs.index_values(n)
    d = -(-(1 << 32) // m)
    fn = ms.BucketFn.div(d)
    say("case autotune m=%d kv=%d n=%d" % (m, kv, n))
    dk, dv = dev(keys), dev(vals) if kv else None
    opt, t = ms.autotune(ms.OP_PAIRS if kv else ms.OP_KEYS, dk, dv, m, fn=fn, reps=2)
    assert t > 0.0
    assert (opt.reorder, opt.waves_per_block, opt.items_per_lane) in MULTI
    ek, ev, eo = oracle.multisplit(keys, m, oracle.DIV, vals=vals if kv else None, divisor=d)
    if kv:
        k, v, o = ms.pairs(dk, dv, m, fn, options=opt)
        np.testing.assert_array_equal(host(v), ev)
    else:
        k, o = ms.keys(dk, m, fn, options=opt)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)


def test_autotune_keeps_untuned_fields_of_base():
    from paper_1701_01189_amd import binding as ms
    n = 300_001
    keys = inputs.uniform_u32(311, n)
    fn = ms.BucketFn.shift_mask(27, 31)
    base = ms.Options(max_chunks=3, prescan=ms.PRESCAN_LANES)
    say("case autotune base max_chunks=3 prescan=lanes")
    opt, _ = ms.autotune(ms.OP_KEYS, dev(keys), None, 32, fn=fn, reps=1, base=base)
    assert opt.max_chunks == 3
    # lane counters need block reordering; other modes fall back to AUTO
    assert opt.prescan == (ms.PRESCAN_LANES if opt.reorder == ms.REORDER_BLOCK
                           else ms.PRESCAN_AUTO)
    ek, _, eo = oracle.multisplit(keys, 32, oracle.SHIFT_MASK, shift=27, mask=31)
    k, o = ms.keys(dev(keys), 32, fn, options=opt)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)


def test_autotune_batched_winner_matches_oracle():
    from paper_1701_01189_amd import binding as ms
    sizes = inputs.batched_sizes(321, 200, 4, 14)
    seg = inputs.segment_offsets(sizes)
    keys, vals = inputs.batched_pairs(321, sizes)
    dseg = torch.from_numpy(seg.astype(np.int64)).cuda()
    fn = ms.BucketFn.shift_mask(8, 63)
    say("case autotune batched instances=%d total=%d" % (len(sizes), len(keys)))
    opt, t = ms.autotune(ms.OP_BATCHED, dev(keys), dev(vals), 64, fn=fn, seg=dseg, reps=2)
    assert t > 0.0
    assert opt.reorder == ms.REORDER_BLOCK
    assert (opt.waves_per_block, opt.items_per_lane, opt.batch_claim) in BATCH
    ek, ev, eo = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    k, v, o, ws = ms.batched(dev(keys), dev(vals), dseg, 64, fn, options=opt)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(v), ev)
    np.testing.assert_array_equal(host(o), eo)
    assert ms.batched_status(ws) == 0


@pytest.mark.parametrize("kv", [False, True])
def test_autotune_radix_winner_matches_oracle(kv):
    from paper_1701_01189_amd import binding as ms
    n = 200_003
    keys = inputs.uniform_u32(331, n)
    keys[::7] = keys[3]  # ties make stability observable
    vals = inputs.index_values(n)
    op = ms.OP_RADIX_SORT_PAIRS if kv else ms.OP_RADIX_SORT
    say("case autotune radix kv=%d n=%d" % (kv, n))
    opt, t = ms.autotune(op, dev(keys), dev(vals) if kv else None, 8, reps=1)
    assert t > 0.0
    assert (opt.reorder, opt.waves_per_block, opt.items_per_lane) in MULTI
    ek, ev = oracle.radix_sort(keys, vals)
    k, v = ms.radix_sort(dev(keys), dev(vals) if kv else None, bits_per_pass=8, options=opt)
    np.testing.assert_array_equal(host(k), ek)
    if kv:
        np.testing.assert_array_equal(host(v), ev)


def test_tuned_options_measures_once_then_reads_the_cache(tmp_path):
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import tuning
    cache = str(tmp_path / "tune.json")
    n = (1 << 19) + 5
    keys = inputs.uniform_u32(341, n)
    fn = ms.BucketFn.shift_mask(28, 15)
    dk = dev(keys)
    say("case tuned_options cache=%s" % cache)
    opt1, e1 = tuning.tuned_options(ms.OP_KEYS, dk, None, 16, fn=fn, cache=cache, reps=1)
    table = json.load(open(cache))
    assert len(table) == 1
    (key, stored), = table.items()
    assert key.startswith("op%d|m16|n2^20|kv0|kind%d|" % (ms.OP_KEYS, ms.BUCKET_SHIFT_MASK))
    assert stored == e1 and stored["ms"] > 0.0
    opt2, e2 = tuning.tuned_options(ms.OP_KEYS, dk, None, 16, fn=fn, cache=cache, reps=1)
    assert e2 == e1
    assert (opt2.reorder, opt2.waves_per_block, opt2.items_per_lane) == \
        (opt1.reorder, opt1.waves_per_block, opt1.items_per_lane)
    ek, _, eo = oracle.multisplit(keys, 16, oracle.SHIFT_MASK, shift=28, mask=15)
    k, o = ms.keys(dk, 16, fn, options=opt2)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("op", ["keys", "batched"])
def test_autotune_skips_a_failing_candidate(op):
    """With test flag bit 1 the first candidate reports failure: the search
    goes on, the winner is another candidate and the operation run with it
    is still exact."""
    from paper_1701_01189_amd import binding as ms
    m = 32
    fn = ms.BucketFn.shift_mask(27, 31)
    base = ms.Options(test_flags=2)
    if op == "keys":
        n = (1 << 20) + 3
        keys = inputs.uniform_u32(61, n)
        dk = dev(keys)
        say("case autotune failing first candidate keys")
        opt, t = ms.autotune(ms.OP_KEYS, dk, None, m, fn=fn, reps=1, base=base)
        assert (opt.reorder, opt.waves_per_block, opt.items_per_lane) in MULTI - {(1, 8, 8)}
        assert opt.test_flags == 0 and t > 0.0
        k, o = ms.keys(dk, m, fn, options=opt)
        ek, _, eo = oracle.multisplit(keys, m, oracle.SHIFT_MASK, shift=27, mask=31)
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)
    else:
        sizes = inputs.batched_sizes(62, 40)
        seg = inputs.segment_offsets(sizes)
        keys, vals = inputs.batched_pairs(62, sizes)
        dk, dv = dev(keys), dev(vals)
        ds = torch.from_numpy(seg.astype(np.int64)).cuda()
        say("case autotune failing first candidate batched")
        opt, t = ms.autotune(ms.OP_BATCHED, dk, dv, m, fn=fn, seg=ds, reps=1, base=base)
        assert (opt.waves_per_block, opt.items_per_lane, opt.batch_claim) in BATCH - {(8, 8, 4)}
        assert opt.test_flags == 0
        k, v, o, _ = ms.batched(dk, dv, ds, m, fn, options=opt)
        ek, ev, eo = oracle.batched(keys, vals, seg, m, oracle.SHIFT_MASK, shift=27, mask=31)
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)
