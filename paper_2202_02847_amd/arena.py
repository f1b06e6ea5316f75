"""Arena layout of work lists: offsets of packed solids (marshalling only, no arithmetic
of the method).

A solid of order P holds P(P+1) reals, an even number, so packing solids back to back
from offset 0 keeps every offset even, as the work-list calls require.
"""
from __future__ import annotations

import numpy as np


def solid_reals(p):
    p = np.asarray(p, dtype=np.int64)
    return p * (p + 1)


def packed_offsets(orders, group_by_order: bool = False):
    """Offsets of solids of the given orders packed back to back; returns (offsets, total).
    group_by_order=True lays the solids out in blocks of equal order (ascending), items
    keeping their relative order inside a block -- convenient when a batched call fills
    each block (one order per call)."""
    orders = np.asarray(orders, dtype=np.int64)
    sizes = solid_reals(orders)
    if not group_by_order:
        ends = np.cumsum(sizes)
        return ends - sizes, int(ends[-1]) if len(ends) else 0
    perm = np.argsort(orders, kind="stable")
    ends = np.cumsum(sizes[perm])
    offs = np.empty_like(sizes)
    offs[perm] = ends - sizes[perm]
    return offs, int(ends[-1]) if len(ends) else 0


def order_blocks(orders, offsets):
    """For solids laid out by packed_offsets(group_by_order=True): a list of
    (order, first offset, item indices) per block."""
    orders = np.asarray(orders)
    out = []
    for p in np.unique(orders):
        idx = np.nonzero(orders == p)[0]
        out.append((int(p), int(np.min(offsets[idx])), idx))
    return out
