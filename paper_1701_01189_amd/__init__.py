"""Stable multisplit for AMD Instinct MI355X (gfx950).

Implements the three-stage multisplit of Ashkiani et al., "GPU Multisplit:
an extended study of a parallel algorithm" (pre-scan, scan, post-scan with
wavefront-ballot ranking and LDS reordering) as hand-written HIP kernels
behind the C ABI in include/multisplit.h.  This package is the thin Python
binding (``binding``), the in-tree build (``build``) and the seeded input
generators (``inputs``).  ``sssp`` is the delta-stepping shortest-path
application of Section 7.2 built on the multisplit.  The native library is loaded on first use.
"""
from .binding import (BUCKET_DIV, BUCKET_LEARNED, BUCKET_SHIFT_MASK, BUCKET_SPLITTERS,
                      MODEL_FLOATS, OP_BATCHED, OP_HISTOGRAM, OP_KEYS, OP_LEARNED_FIT, OP_PAIRS, OP_RADIX_SORT,
                      OP_RADIX_SORT_PAIRS,
                      PRESCAN_AUTO, PRESCAN_BALLOT, PRESCAN_LANES,
                      REORDER_AUTO, REORDER_BLOCK, REORDER_NONE, REORDER_WAVE, BucketFn,
                      MultisplitError, Options, batched, batched_status, copy_u32, histogram, keys, learned_fit, pairs,
                      radix_sort, sssp, sssp_workspace_size,
                      workspace_size)
