"""GPU parity of range buckets: binary search over splitters and the learned
bucket identifier (model prediction + exact correction) against the oracle.

The learned path must give exactly the upper-bound bucket of every key, so
its multisplit output is compared bit-exactly with the oracle's splitter
multisplit.  With the CPU-fitted model loaded, the GPU's count of raw-model
mispredictions must equal the oracle's count exactly (same float32 fused
multiply-add evaluation).  The GPU fit itself is compared with the CPU fit
parameter by parameter (relative 1e-5) and by misprediction rate (within 0.1
percentage points): the two sum in different orders.
"""
import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def devf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def say(*a):
    print(*a, flush=True)


def lognormal_setup(n, fit_n=1 << 18):
    sample = inputs.lognormal_u32(1031, 1 << 16)
    spl = inputs.quantile_splitters(sample, 256)
    fit = inputs.lognormal_u32(1032, fit_n)
    keys = inputs.lognormal_u32(103, n)
    return keys, spl, fit


SHAPES = [(1, 8, 8), (1, 4, 8), (1, 16, 8), (2, 8, 8), (3, 8, 8)]


def test_learned_and_binary_search_match_oracle_with_cpu_model():
    from paper_1701_01189_amd import binding as ms
    n = (1 << 22) + 333
    keys, spl, fit = lognormal_setup(n)
    model = oracle.learned_fit(fit, spl, 256)
    ek, _, eo = oracle.multisplit(keys, 256, oracle.SPLITTERS, splitters=spl)
    _, emiss = oracle.learned_bucket_ids(model, spl, 256, keys)
    dk, ds, dm = dev(keys), dev(spl), devf(model)
    for shape in SHAPES:
        say("case splitters shape=%s" % (shape,))
        k, o = ms.keys(dk, 256, ms.BucketFn.splitter(ds), options=ms.Options(*shape))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)
        say("case learned shape=%s" % (shape,))
        miss = torch.zeros(1, dtype=torch.int64, device="cuda")
        k, o = ms.keys(dk, 256, ms.BucketFn.learned(ds, dm),
                       options=ms.Options(*shape, mispredicts=miss))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)
        assert int(miss.item()) == emiss


def test_learned_pairs_small_m_and_duplicates():
    from paper_1701_01189_amd import binding as ms
    for m in (2, 3, 17, 100, 255):
        n = 50_001 + m
        keys = inputs.uniform_u32(300 + m, n)
        vals = inputs.index_values(n)
        spl = np.sort(inputs.uniform_u32(400 + m, m - 1))
        if m > 10:
            spl[3:9] = spl[3]  # zero-width buckets
            spl = np.sort(spl)
        keys[:m - 1] = spl   # keys equal to splitters go up
        model = oracle.learned_fit(inputs.uniform_u32(500 + m, 20_000), spl, m)
        ek, ev, eo = oracle.multisplit(keys, m, oracle.SPLITTERS, vals=vals, splitters=spl)
        _, emiss = oracle.learned_bucket_ids(model, spl, m, keys)
        say("case learned pairs m=%d" % m)
        miss = torch.zeros(1, dtype=torch.int64, device="cuda")
        k, v, o = ms.pairs(dev(keys), dev(vals), m, ms.BucketFn.learned(dev(spl), devf(model)),
                           options=ms.Options(mispredicts=miss))
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(v), ev)
        np.testing.assert_array_equal(host(o), eo)
        assert int(miss.item()) == emiss


def test_gpu_fit_against_cpu_fit():
    from paper_1701_01189_amd import binding as ms
    n = 1 << 20
    keys, spl, fit = lognormal_setup(1 << 20, fit_n=1 << 20)
    cpu = oracle.learned_fit(fit, spl, 256)
    say("case gpu fit 2^20")
    gm = ms.learned_fit(dev(fit), dev(spl), 256)
    torch.cuda.synchronize()
    gpu = gm.cpu().numpy()
    np.testing.assert_allclose(gpu, cpu, rtol=1e-5, atol=1e-12)
    _, miss_cpu = oracle.learned_bucket_ids(cpu, spl, 256, keys)
    _, miss_gpu = oracle.learned_bucket_ids(gpu, spl, 256, keys)
    assert abs(miss_cpu - miss_gpu) / n <= 0.001
    # deterministic: a second fit is bit-identical
    gm2 = ms.learned_fit(dev(fit), dev(spl), 256)
    np.testing.assert_array_equal(gm2.cpu().numpy(), gpu)
    # and it is a usable model: the multisplit stays exact
    ek, _, eo = oracle.multisplit(keys, 256, oracle.SPLITTERS, splitters=spl)
    k, o = ms.keys(dev(keys), 256, ms.BucketFn.learned(dev(spl), gm))
    np.testing.assert_array_equal(host(k), ek)


def test_gpu_fit_with_labels():
    """Labels passed in: the upper-bound labels give the GPU fit without
    labels bit for bit; other labels (top byte of the key) match the
    oracle's fit to the same labels within the fit tolerance; no splitters
    are needed then."""
    from paper_1701_01189_amd import binding as ms
    keys, spl, fit = lognormal_setup(1 << 16, fit_n=(1 << 18) + 77)
    ds, dfit = dev(spl), dev(fit)
    say("case gpu fit with labels")
    ub = np.searchsorted(spl, fit, side="right").astype(np.uint32)
    g0 = ms.learned_fit(dfit, ds, 256).cpu().numpy()
    g1 = ms.learned_fit(dfit, ds, 256, labels=dev(ub)).cpu().numpy()
    np.testing.assert_array_equal(g0, g1)
    lab = (fit >> np.uint32(24)).astype(np.uint32)
    cpu = oracle.learned_fit(fit, spl, 256, labels=lab)
    g2 = ms.learned_fit(dfit, None, 256, labels=dev(lab)).cpu().numpy()
    np.testing.assert_allclose(g2, cpu, rtol=1e-5, atol=1e-12)


def test_gpu_fit_degenerate_samples():
    """All sample keys equal (zero key range), two distinct keys, and the
    saturated top key only: the GPU fit matches the oracle's."""
    from paper_1701_01189_amd import binding as ms
    spl = np.sort(inputs.uniform_u32(61, 255))
    for name, fit in (("equal", np.full(5000, 123456789, np.uint32)),
                      ("two", np.array([7, 0xFFFFFFFF] * 3000, np.uint32)),
                      ("top", np.full(4097, 0xFFFFFFFF, np.uint32)),
                      ("one", np.array([0], np.uint32))):
        say("case gpu fit degenerate %s" % name)
        cpu = oracle.learned_fit(fit, spl, 256)
        gpu = ms.learned_fit(dev(fit), dev(spl), 256).cpu().numpy()
        np.testing.assert_allclose(gpu, cpu, rtol=1e-5, atol=1e-12)


def test_range_2e27_lognormal_learned_full_size():
    """n = 2^27 lognormal(20, 2) saturated keys (seed 103), m = 256 buckets at
    quantiles of a 2^16-key sample (seed 1031); model fit on the GPU from 2^20
    keys (seed 1032).  Learned and binary-search outputs equal the oracle."""
    from paper_1701_01189_amd import binding as ms
    n = 1 << 27
    keys, spl, fit = lognormal_setup(n, fit_n=1 << 20)
    ek, _, eo = oracle.multisplit(keys, 256, oracle.SPLITTERS, splitters=spl)
    dk, ds = dev(keys), dev(spl)
    say("case range 2^27 fit")
    gm = ms.learned_fit(dev(fit), ds, 256)
    say("case range 2^27 learned")
    k, o = ms.keys(dk, 256, ms.BucketFn.learned(ds, gm))
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)
    say("case range 2^27 binary search")
    k, o = ms.keys(dk, 256, ms.BucketFn.splitter(ds))
    np.testing.assert_array_equal(host(k), ek)
    np.testing.assert_array_equal(host(o), eo)


@pytest.mark.parametrize("kv", [False, True])
def test_kept_bucket_ids_match_oracle(kv):
    """keep_bucket_ids: the pre-scan stores each key's bucket id and the
    post-scan reads it; the output is the same unique stable multisplit, for
    block (several tile shapes), wave-level and no reordering, on lognormal
    keys over 256 range buckets and on uniform keys over 50 splitters (one
    bucket per lane path); several tiles per chunk and a ragged tail."""
    from paper_1701_01189_amd import binding as ms
    n = (1 << 21) + 4097
    keys, spl, fit = lognormal_setup(n)
    model = oracle.learned_fit(fit, spl, 256)
    vals = inputs.index_values(n) if kv else None
    ek, ev, eo = oracle.multisplit(keys, 256, oracle.SPLITTERS, vals=vals, splitters=spl)
    dk, ds, dm = dev(keys), dev(spl), devf(model)
    dv = dev(vals) if kv else None
    # (16 x 16 key-value tiles with their bucket ids do not fit in LDS)
    shapes = [(1, 8, 8), (1, 16, 8), (2, 8, 8), (3, 8, 8)] + ([] if kv else [(1, 16, 16)])
    for shape in shapes:
        for name, fn in (("splitters", ms.BucketFn.splitter(ds)),
                         ("learned", ms.BucketFn.learned(ds, dm))):
            say("case kept ids %s kv=%s shape=%s" % (name, kv, shape))
            opt = ms.Options(*shape, max_chunks=37, keep_bucket_ids=1)
            if kv:
                k, v, o = ms.pairs(dk, dv, 256, fn, options=opt)
                np.testing.assert_array_equal(host(v), ev)
            else:
                k, o = ms.keys(dk, 256, fn, options=opt)
            np.testing.assert_array_equal(host(k), ek)
            np.testing.assert_array_equal(host(o), eo)
    # m = 50 (a bucket per lane, 49 splitters), uniform keys
    m = 50
    ukeys = inputs.uniform_u32(151, n)
    uspl = np.sort(inputs.uniform_u32(152, m - 1))
    uvals = inputs.index_values(n) if kv else None
    ek, ev, eo = oracle.multisplit(ukeys, m, oracle.SPLITTERS, vals=uvals, splitters=uspl)
    dk, ds = dev(ukeys), dev(uspl)
    dv = dev(uvals) if kv else None
    for shape in [(1, 8, 8), (2, 8, 8), (3, 8, 8)]:
        say("case kept ids m=50 kv=%s shape=%s" % (kv, shape))
        opt = ms.Options(*shape, keep_bucket_ids=1)
        if kv:
            k, v, o = ms.pairs(dk, dv, m, ms.BucketFn.splitter(ds), options=opt)
            np.testing.assert_array_equal(host(v), ev)
        else:
            k, o = ms.keys(dk, m, ms.BucketFn.splitter(ds), options=opt)
        np.testing.assert_array_equal(host(k), ek)
        np.testing.assert_array_equal(host(o), eo)


def test_kept_bucket_ids_count_the_same_mispredictions():
    """With kept ids the raw-model mispredictions are counted by the
    pre-scan: the count equals the oracle's, as without kept ids."""
    from paper_1701_01189_amd import binding as ms
    n = (1 << 20) + 77
    keys, spl, fit = lognormal_setup(n)
    model = oracle.learned_fit(fit, spl, 256)
    _, emiss = oracle.learned_bucket_ids(model, spl, 256, keys)
    dk, ds, dm = dev(keys), dev(spl), devf(model)
    for keep in (0, 1):
        miss = torch.zeros(1, dtype=torch.int64, device="cuda")
        ms.keys(dk, 256, ms.BucketFn.learned(ds, dm),
                options=ms.Options(mispredicts=miss, keep_bucket_ids=keep))
        torch.cuda.synchronize()
        assert int(miss.item()) == int(emiss), (keep, int(miss.item()), int(emiss))
