"""The byte model the benchmark prices every rate with, pinned to the
speed-of-light figures the paper prints (Section 6.2.2): its rates for the
K40c (288 GB/s) and GTX 1080 (320 GB/s) follow from 3 four-byte accesses per
key and 5 per key-value pair (tests/golden/speed_of_light.txt)."""
import os

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "speed_of_light.txt")


def rows():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            gpu, bw, keys, pairs = line.split()
            out.append((gpu, float(bw), float(keys), float(pairs)))
    return out


def test_golden_has_both_gpus():
    assert [r[0] for r in rows()] == ["K40c", "GTX1080"]


def test_byte_model_gives_the_printed_rates():
    for gpu, bw, keys, pairs in rows():
        # the paper prints its rates to about three significant figures
        assert abs(bench.sol_rate(bw, kv=False) - keys) < 0.1, gpu
        assert abs(bench.sol_rate(bw, kv=True) - pairs) < 0.1, gpu


def test_post_scan_share_and_gate():
    # the pre-scan reads the key once; the post-scan moves the rest
    assert bench.BYTES_PER_KEY == bench.POST_BYTES_PER_KEY + 4
    assert bench.BYTES_PER_PAIR == bench.POST_BYTES_PER_PAIR + 4
    # 60 % of 8 TB/s at 12 B/key is 400 Gkeys/s
    assert abs(bench.GATE_FRAC * bench.sol_rate(bench.HBM_PEAK_GBPS, kv=False) - 400.0) < 1e-9
