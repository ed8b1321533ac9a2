"""GPU parity of the batched persistent multisplit against the oracle applied
to every instance on its own, bit-exact (keys, values, per-instance offsets).

Also: capture into a HIP graph and replay several times with eager work in
between (every replay is checked), and the bounded-wait failure path forced
from the host (ready flags never raised, a tiny poll limit: every wait
expires, the kernel still finishes and the status reports the timeout).
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


def instances(seed, num, lo, hi, zero_every=0):
    sizes = inputs.batched_sizes(seed, num, lo, hi)
    if zero_every:
        sizes[::zero_every] = 0
    seg = inputs.segment_offsets(sizes)
    keys, vals = inputs.batched_pairs(seed, sizes)
    return sizes, seg, keys, vals


def dseg(seg):
    return torch.from_numpy(seg.astype(np.int64)).cuda()


@pytest.mark.parametrize("shape", [(8, 8, 1), (8, 4, 1), (8, 8, 4), (8, 4, 16)])
def test_batched_shift_mask_vs_oracle(shape):
    from paper_1701_01189_amd import binding as ms
    sizes, seg, keys, vals = instances(11, 300, 0, 15, zero_every=37)
    ek, ev, eo = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    say("case batched shift shape=%s total=%d" % (shape, len(keys)))
    opt = ms.Options(waves_per_block=shape[0], items_per_lane=shape[1], batch_claim=shape[2])
    k, v, o, ws = ms.batched(dev(keys), dev(vals), dseg(seg), 64, ms.BucketFn.shift_mask(8, 63),
                             options=opt)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(v), ev)
    np.testing.assert_array_equal(host(o), eo)
    assert ms.batched_status(ws) == 0


@pytest.mark.parametrize("m", [1, 2, 7, 200, 256])
def test_batched_other_kinds_and_keys_only(m):
    from paper_1701_01189_amd import binding as ms
    sizes, seg, keys, vals = instances(50 + m, 120, 0, 14, zero_every=29)
    d = min(-(-(1 << 32) // m), 0xFFFFFFFF)
    if m > 1:
        say("case batched div m=%d" % m)
        ek, ev, eo = oracle.batched(keys, vals, seg, m, oracle.DIV, divisor=d)
        k, v, o, ws = ms.batched(dev(keys), dev(vals), dseg(seg), m, ms.BucketFn.div(d))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)
    spl = np.sort(inputs.uniform_u32(7 + m, max(m - 1, 1)))[:m - 1]
    ek, _, eo = oracle.batched(keys, None, seg, m, oracle.SPLITTERS, splitters=spl)
    ds = dev(spl if m > 1 else np.zeros(1, np.uint32))
    say("case batched splitters keys-only m=%d" % m)
    k, _, o, ws = ms.batched(dev(keys), None, dseg(seg), m, ms.BucketFn.splitter(ds))
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)
    if m > 1:
        model = oracle.learned_fit(inputs.uniform_u32(9 + m, 4096), spl, m)
        dm = torch.from_numpy(model).cuda()
        say("case batched learned m=%d" % m)
        k, _, o, ws = ms.batched(dev(keys), None, dseg(seg), m, ms.BucketFn.learned(ds, dm))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)


def test_batched_4096_instances_m64_full_size():
    """4096 instances, sizes log-uniform in [2^8, 2^20] (seed 104), uint32 keys
    uniform (seed 104000 + i) and values = index within the instance, m = 64,
    f(k) = (k >> 8) & 63."""
    from paper_1701_01189_amd import binding as ms
    sizes, seg, keys, vals = instances(104, 4096, 8, 20)
    say("case batched 4096 total=%d" % len(keys))
    ek, ev, eo = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    k, v, o, ws = ms.batched(dev(keys), dev(vals), dseg(seg), 64, ms.BucketFn.shift_mask(8, 63))
    np.testing.assert_array_equal(host(o), eo)
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(v), ev)
    assert ms.batched_status(ws) == 0


def test_batched_graph_capture_replays():
    from paper_1701_01189_amd import binding as ms
    sizes, seg, keys, vals = instances(21, 500, 4, 16)
    ek, ev, eo = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    dk, dv, ds = dev(keys), dev(vals), dseg(seg)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    off = torch.empty(len(sizes) * 65, dtype=torch.int32, device="cuda")
    need = ms.workspace_size(ms.OP_BATCHED, len(keys), 64, len(sizes))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    fn = ms.BucketFn.shift_mask(8, 63)
    # eager warm-up on the side stream used for capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ms.batched(dk, dv, ds, 64, fn, keys_out=ko, vals_out=vo, offsets=off, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("case batched graph capture")
    with torch.cuda.graph(g):
        ms.batched(dk, dv, ds, 64, fn, keys_out=ko, vals_out=vo, offsets=off, ws=ws)
    for rep in range(4):
        ko.zero_()
        vo.zero_()
        off.zero_()
        torch.cuda.synchronize()
        say("case batched graph replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(ko), ek)
        np.testing.assert_array_equal(host(vo), ev)
        np.testing.assert_array_equal(host(off), eo)
        assert ms.batched_status(ws) == 0


def test_batched_wait_timeout_is_reported():
    from paper_1701_01189_amd import binding as ms
    sizes, seg, keys, vals = instances(31, 40, 6, 12)
    say("case batched forced timeout")
    opt = ms.Options(spin_limit=8, test_flags=1)
    k, v, o, ws = ms.batched(dev(keys), dev(vals), dseg(seg), 64, ms.BucketFn.shift_mask(8, 63),
                             options=opt)
    torch.cuda.synchronize()
    assert ms.batched_status(ws) == -5
    # the next normal call on the same workspace succeeds and is exact
    ek, ev, eo = oracle.batched(keys, vals, seg, 64, oracle.SHIFT_MASK, shift=8, mask=63)
    k, v, o, ws2 = ms.batched(dev(keys), dev(vals), dseg(seg), 64, ms.BucketFn.shift_mask(8, 63),
                              ws=ws)
    assert ms.batched_status(ws) == 0
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(v), ev)
