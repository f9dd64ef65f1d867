"""Wave orders for uneven work.

Chains of uneven length go to slots sorted by decreasing length
(brng_sort_by_length); LDA documents of uneven size can be handed to waves
in order of decreasing work (the descriptor's perm for LDA), so that the
largest start first and the launch does not end on a tail of lone large
documents.  Neither order changes a result (units are keyed by chain block
or by document, not by wave).
"""
from __future__ import annotations

import numpy as np

from . import binding as b

# Per-sweep cost of a document on MI355X in SIMD cycles, measured on
# homogeneous runs (16,384 documents x 100 sweeps): about 1,320 + 14.7 K for
# the gamma rounds, normalisation and bookkeeping, plus 6 per token for the
# multinomial; in units of one token.
_FIXED, _PER_COMPONENT = 220.0, 2.45


def doc_order(offsets, ntok) -> np.ndarray:
    """Documents by decreasing estimated work (stable), as int32."""
    off = np.asarray(offsets, dtype=np.int64)
    K = np.diff(off)
    work = np.rint(_FIXED + _PER_COMPONENT * K + np.asarray(ntok, dtype=np.float64))
    return b.brng_sort_by_length(np.minimum(work, 2 ** 31 - 1).astype(np.int32))
