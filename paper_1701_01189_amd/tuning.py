"""Persistent cache of autotuned options (JSON), keyed by operation, bucket
count, size class, key-only/key-value, bucket kind and device architecture.
The timing itself is ms_autotune in the native library."""
from __future__ import annotations

import json
import os

from . import binding as ms

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "multisplit_gfx950_tune.json")


def _key(op, n, m, kv, kind, num, ids=0):
    ncls = max(0, int(n - 1).bit_length())
    return "op%d|m%d|n2^%d|kv%d|kind%d|inst%d|ids%d|gfx950" % (
        op, m, ncls, int(kv), kind, max(0, int(num).bit_length()), int(ids))


def tuned_options(op, keys_in, vals_in, m, fn=None, seg=None, cache=None, reps=3, retune=False,
                  keep_bucket_ids=0):
    """Options for this problem shape: from the cache, else measured with
    ms_autotune on these inputs and stored."""
    path = cache or os.environ.get("MS_TUNE_CACHE", DEFAULT_CACHE)
    num = seg.numel() - 1 if seg is not None else 0
    kind = fn.kind if fn is not None else 0
    key = _key(op, keys_in.numel(), m, vals_in is not None, kind, num, keep_bucket_ids)
    table = {}
    if os.path.exists(path):
        try:
            table = json.load(open(path))
        except ValueError:
            table = {}
    if not retune and key in table:
        e = table[key]
        return ms.Options(reorder=e["reorder"], waves_per_block=e["waves_per_block"],
                          items_per_lane=e["items_per_lane"], batch_claim=e["batch_claim"],
                          prescan=e.get("prescan", 0), keep_bucket_ids=keep_bucket_ids), e
    base = ms.Options(keep_bucket_ids=keep_bucket_ids) if keep_bucket_ids else None
    opt, t = ms.autotune(op, keys_in, vals_in, m, fn=fn, seg=seg, reps=reps, base=base)
    e = {"reorder": opt.reorder, "waves_per_block": opt.waves_per_block,
         "items_per_lane": opt.items_per_lane, "batch_claim": opt.batch_claim,
         "prescan": opt.prescan, "ms": t}
    table[key] = e
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return opt, e
