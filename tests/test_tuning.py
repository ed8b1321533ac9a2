"""Host logic of the autotune cache (tuning.py) and the autotuner's argument
checks, without a GPU: the timing call is replaced by a stub, so these check
the cache's keying, hits, misses and recovery from a damaged file."""
import ctypes
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")


class Counting:
    """Stands in for binding.autotune: returns fixed options and counts calls."""

    def __init__(self, ms, **fields):
        self.ms, self.fields, self.calls = ms, fields, []

    def __call__(self, op, keys_in, vals_in, m, fn=None, seg=None, reps=3, base=None):
        self.calls.append((op, keys_in.numel(), vals_in is not None, m, reps))
        return self.ms.Options(**self.fields), 0.125


def keys(n):
    return torch.zeros(n, dtype=torch.int32)


def test_cache_key_size_classes():
    from paper_1701_01189_amd import tuning
    assert tuning._key(0, 1 << 20, 32, False, 0, 0) == "op0|m32|n2^20|kv0|kind0|inst0|ids0|gfx950"
    assert tuning._key(0, (1 << 20) + 1, 32, False, 0, 0).split("|")[2] == "n2^21"
    assert tuning._key(0, (1 << 19) + 1, 32, False, 0, 0).split("|")[2] == "n2^20"
    assert tuning._key(1, 1, 256, True, 2, 0) == "op1|m256|n2^0|kv1|kind2|inst0|ids0|gfx950"
    assert tuning._key(2, 1000, 64, True, 0, 4096).endswith("|inst13|ids0|gfx950")
    # every field separates entries
    base = tuning._key(1, 5000, 32, True, 1, 0)
    for other in (tuning._key(0, 5000, 32, True, 1, 0), tuning._key(1, 5000, 16, True, 1, 0),
                  tuning._key(1, 50000, 32, True, 1, 0), tuning._key(1, 5000, 32, False, 1, 0),
                  tuning._key(1, 5000, 32, True, 0, 0), tuning._key(1, 5000, 32, True, 1, 3)):
        assert other != base


def test_miss_measures_and_stores_then_hit_reads(tmp_path, monkeypatch):
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import tuning
    stub = Counting(ms, reorder=2, waves_per_block=4, items_per_lane=16, prescan=1)
    monkeypatch.setattr(ms, "autotune", stub)
    cache = str(tmp_path / "sub" / "tune.json")
    fn = ms.BucketFn.div(1 << 27)
    opt, e = tuning.tuned_options(ms.OP_KEYS, keys(3000), None, 32, fn=fn, cache=cache, reps=2)
    assert stub.calls == [(ms.OP_KEYS, 3000, False, 32, 2)]
    assert (opt.reorder, opt.waves_per_block, opt.items_per_lane, opt.prescan) == (2, 4, 16, 1)
    table = json.load(open(cache))
    assert table == {"op0|m32|n2^12|kv0|kind1|inst0|ids0|gfx950": e}
    assert e["ms"] == 0.125
    opt2, e2 = tuning.tuned_options(ms.OP_KEYS, keys(2100), None, 32, fn=fn, cache=cache)
    assert len(stub.calls) == 1 and e2 == e  # same size class: read from the cache
    assert (opt2.reorder, opt2.waves_per_block, opt2.items_per_lane, opt2.prescan) == \
        (2, 4, 16, 1)
    tuning.tuned_options(ms.OP_KEYS, keys(5000), None, 32, fn=fn, cache=cache)
    assert len(stub.calls) == 2  # next size class: measured
    assert len(json.load(open(cache))) == 2
    tuning.tuned_options(ms.OP_KEYS, keys(3000), None, 32, fn=fn, cache=cache, retune=True)
    assert len(stub.calls) == 3


def test_entries_without_prescan_and_damaged_files(tmp_path, monkeypatch):
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import tuning
    stub = Counting(ms, reorder=1, waves_per_block=8, items_per_lane=8, batch_claim=4)
    monkeypatch.setattr(ms, "autotune", stub)
    cache = tmp_path / "tune.json"
    key = tuning._key(ms.OP_PAIRS, 4096, 8, True, 0, 0)
    # an entry written before the pre-scan choice was tuned has no "prescan"
    cache.write_text(json.dumps({key: {"reorder": 3, "waves_per_block": 8, "items_per_lane": 8,
                                       "batch_claim": 0, "ms": 1.0}}))
    opt, _ = tuning.tuned_options(ms.OP_PAIRS, keys(4096), keys(4096), 8, cache=str(cache))
    assert stub.calls == [] and opt.reorder == 3 and opt.prescan == 0
    cache.write_text("{not json")
    opt, e = tuning.tuned_options(ms.OP_PAIRS, keys(4096), keys(4096), 8, cache=str(cache))
    assert len(stub.calls) == 1 and opt.batch_claim == 4
    assert json.load(open(cache)) == {key: e}


def test_cache_path_from_environment(tmp_path, monkeypatch):
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import tuning
    stub = Counting(ms, reorder=1, waves_per_block=8, items_per_lane=8)
    monkeypatch.setattr(ms, "autotune", stub)
    path = tmp_path / "env_tune.json"
    monkeypatch.setenv("MS_TUNE_CACHE", str(path))
    seg = torch.from_numpy(np.array([0, 10, 30], dtype=np.int64))
    tuning.tuned_options(ms.OP_BATCHED, keys(30), keys(30), 64, seg=seg)
    assert list(json.load(open(path))) == [tuning._key(ms.OP_BATCHED, 30, 64, True, 0, 2)]


def test_autotune_rejects_bad_arguments_on_the_host():
    from paper_1701_01189_amd import binding as ms
    from paper_1701_01189_amd import build
    if build.stale():
        build.build(force=True)
    L = ms.lib()
    best = ms.OptionsC()
    t = ctypes.c_float(0.0)
    fn = ms.BucketFnC(0, 27, 31, 0, None, None)
    k, o, w = ctypes.c_void_p(0x1000000), ctypes.c_void_p(0x9000000), ctypes.c_void_p(0x20000000)

    def call(op, reps, best_ptr):
        return L.ms_autotune(op, k, None, o, None, None, 0, 1000, 32, ctypes.byref(fn), w,
                             1 << 20, reps, None, best_ptr, ctypes.byref(t), None)

    invalid = -1
    assert call(ms.OP_KEYS, 1, None) == invalid              # nowhere to write the winner
    assert call(ms.OP_KEYS, 0, ctypes.byref(best)) == invalid
    assert call(ms.OP_KEYS, 1001, ctypes.byref(best)) == invalid
    assert call(ms.OP_LEARNED_FIT, 1, ctypes.byref(best)) == invalid
    assert call(ms.OP_HISTOGRAM, 1, ctypes.byref(best)) == invalid
    assert call(99, 1, ctypes.byref(best)) == invalid
