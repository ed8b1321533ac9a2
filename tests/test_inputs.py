"""Checks of the seeded input generators (runs without a GPU)."""
import math

import numpy as np

from paper_1701_01189_amd import inputs


def test_splitmix64_published_vectors():
    # Reference outputs of SplitMix64 (Steele, Lea, Flood 2014) for seeds 0
    # and 1234567, as printed by the authors' reference implementation.
    assert int(inputs.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF
    assert [int(x) for x in inputs.splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_counter_based_slices():
    a = inputs.splitmix64(9, 1000)
    b = inputs.splitmix64(9, 300, start=700)
    np.testing.assert_array_equal(a[700:], b)
    np.testing.assert_array_equal(inputs.uniform_u32(5, 10), inputs.uniform_u32(5, 20)[:10])


def test_uniform_chi_square():
    k = inputs.uniform_u32(100, 1 << 20)
    cnt = np.bincount(k >> np.uint32(24), minlength=256)
    e = len(k) / 256
    chi2 = float(np.sum((cnt - e) ** 2 / e))
    assert 180 < chi2 < 340  # 255 dof, well inside 6 sigma


def test_lognormal_saturation_fraction():
    k = inputs.lognormal_u32(103, 1 << 20)
    frac = float(np.mean(k == 0xFFFFFFFF))
    z = (math.log(2.0 ** 32) - 20.0) / 2.0
    want = 0.5 * math.erfc(z / math.sqrt(2.0))  # P(exp(20 + 2Z) >= 2^32)
    assert abs(frac - want) < 0.002


def test_binomial_buckets_mean_and_empty_count():
    m, n = 256, 1 << 18
    k = inputs.skewed_bucket_keys(7, n, m, "binomial")
    b = k >> np.uint32(24)
    assert abs(float(np.mean(b)) - 127.5) < 0.1
    # expected number of empty buckets: sum_k (1 - C(255,k)/2^255)^n
    exp_empty = sum((1.0 - math.comb(255, j) / 2.0 ** 255) ** n for j in range(256))
    got = 256 - len(np.unique(b))
    assert abs(got - exp_empty) < 6


def test_alpha_uniform_and_batched_sizes():
    k = inputs.skewed_bucket_keys(8, 1 << 18, 256, "alpha", alpha=0.25)
    cnt = np.bincount(k >> np.uint32(24), minlength=256)
    assert 0.74 < cnt.max() / len(k) < 0.77
    s = inputs.batched_sizes(104, 4096)
    assert s.min() >= 256 and s.max() <= 1 << 20
    # log-uniform: mean of log2 size ~ 14
    assert abs(float(np.mean(np.log2(s))) - 14.0) < 0.2
    seg = inputs.segment_offsets(s)
    assert seg[0] == 0 and seg[-1] == s.sum()


def test_quantile_splitters():
    s = inputs.uniform_u32(3, 1 << 16)
    spl = inputs.quantile_splitters(s, 256)
    srt = np.sort(s)
    assert len(spl) == 255 and np.all(np.diff(spl.astype(np.int64)) >= 0)
    assert spl[0] == srt[256] and spl[-1] == srt[255 * 256]
