"""GPU parity of the device-wide histogram (Section 7.3) against the oracle,
bit-exact: even bins (shift/mask, delta), range bins (splitters, learned),
both pre-scan counting methods and every reordering mode's pre-scan, ragged
sizes, empty input, all keys in one bin, and the paper's size (2^25) and the
benchmark's (2^28) in full."""
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


def cases(m, seed):
    """(name, gpu BucketFn, oracle kind, oracle kwargs, kept tensors)."""
    from paper_1701_01189_amd import binding as ms
    out = []
    r = (m - 1).bit_length()
    if m & (m - 1) == 0:
        s = 32 - r if r else 0
        out.append(("shift", ms.BucketFn.shift_mask(s, m - 1), oracle.SHIFT_MASK,
                    dict(shift=s, mask=m - 1), None))
    if m > 1:
        d = min(-(-(1 << 32) // m), 0xFFFFFFFF)
        out.append(("div", ms.BucketFn.div(d), oracle.DIV, dict(divisor=d), None))
    spl = np.sort(inputs.uniform_u32(seed + 1, max(m - 1, 1)))[:m - 1]
    ds = dev(spl if m > 1 else np.zeros(1, np.uint32))
    out.append(("splitters", ms.BucketFn.splitter(ds), oracle.SPLITTERS, dict(splitters=spl), ds))
    if m > 1:
        model = oracle.learned_fit(inputs.uniform_u32(seed + 2, 1 << 14), spl, m)
        dm = torch.from_numpy(model).cuda()
        out.append(("learned", ms.BucketFn.learned(ds, dm), oracle.SPLITTERS,
                    dict(splitters=spl), (ds, dm)))
    return out


@pytest.mark.parametrize("opt", [(0, 0), (1, 1), (1, 2), (2, 0), (3, 0)])  # (reorder, prescan)
def test_histogram_vs_oracle(opt):
    from paper_1701_01189_amd import binding as ms
    for i, (n, m) in enumerate([(0, 4), (1, 1), (63, 2), (4097, 33), (100003, 64),
                                (70001, 200), (262147, 256), (1 << 20, 8)]):
        keys = inputs.uniform_u32(700 + i, n)
        for name, fn, kind, kw, _keep in cases(m, 40 + i):
            say("case hist n=%d m=%d %s opt=%s" % (n, m, name, opt))
            h = ms.histogram(dev(keys), m, fn, options=ms.Options(reorder=opt[0], prescan=opt[1]))
            np.testing.assert_array_equal(host(h), oracle.histogram(keys, m, kind, **kw))


def test_histogram_one_bin_and_skew():
    from paper_1701_01189_amd import binding as ms
    n = 300_001
    keys = (inputs.uniform_u32(9, n) & np.uint32(0x00FFFFFF)) | np.uint32(0x7B000000)
    for m, shift in ((256, 24), (32, 27), (2, 31)):
        say("case hist one-bin m=%d" % m)
        h = host(ms.histogram(dev(keys), m, ms.BucketFn.shift_mask(shift, m - 1)))
        np.testing.assert_array_equal(h, oracle.histogram(keys, m, oracle.SHIFT_MASK,
                                                          shift=shift, mask=m - 1))
        assert h.sum() == n
    for dist in ("binomial", "alpha"):
        keys = inputs.skewed_bucket_keys(12, 1 << 21, 256, dist)
        say("case hist skew %s" % dist)
        h = host(ms.histogram(dev(keys), 256, ms.BucketFn.shift_mask(24, 255)))
        np.testing.assert_array_equal(h, oracle.histogram(keys, 256, oracle.SHIFT_MASK,
                                                          shift=24, mask=255))


@pytest.mark.parametrize("m", [2, 32, 256])
def test_histogram_full_sizes(m):
    """n = 2^25 (the paper's histogram size) and 2^28 uniform keys, even bins;
    n = 2^25 range bins over m-1 random splitters."""
    from paper_1701_01189_amd import binding as ms
    r = (m - 1).bit_length()
    for n, seed in ((1 << 25, 110), (1 << 28, 111)):
        keys = inputs.uniform_u32(seed, n)
        say("case hist even n=%d m=%d" % (n, m))
        h = host(ms.histogram(dev(keys), m, ms.BucketFn.shift_mask(32 - r, m - 1)))
        np.testing.assert_array_equal(h, oracle.histogram(keys, m, oracle.SHIFT_MASK,
                                                          shift=32 - r, mask=m - 1))
    keys = inputs.uniform_u32(112, 1 << 25)
    spl = np.sort(inputs.uniform_u32(113, m - 1))
    say("case hist range n=2^25 m=%d" % m)
    h = host(ms.histogram(dev(keys), m, ms.BucketFn.splitter(dev(spl))))
    np.testing.assert_array_equal(h, oracle.histogram(keys, m, oracle.SPLITTERS, splitters=spl))


def test_histogram_graph_replays():
    """The call captured in a HIP graph and replayed several times, with eager
    work in between; every replay is checked."""
    from paper_1701_01189_amd import binding as ms
    n, m = 500_003, 64
    keys = inputs.uniform_u32(120, n)
    ref = oracle.histogram(keys, m, oracle.SHIFT_MASK, shift=26, mask=63)
    dk = dev(keys)
    fn = ms.BucketFn.shift_mask(26, 63)
    hist = torch.empty(m, dtype=torch.int32, device="cuda")
    ws = torch.empty(ms.workspace_size(ms.OP_HISTOGRAM, n, m), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ms.histogram(dk, m, fn, hist=hist, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("case hist graph capture")
    with torch.cuda.graph(g):
        ms.histogram(dk, m, fn, hist=hist, ws=ws)
    for rep in range(4):
        hist.fill_(-1)
        ws.zero_()
        torch.cuda.synchronize()
        say("case hist graph replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(hist), ref)
