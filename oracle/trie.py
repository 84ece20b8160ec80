"""Packed linearised tries in the layout of Sec. IV (test infrastructure only).

The trie dispatches on chunks taken from the least significant end.  In the
linear array t, a branch node at index k stores in t[k + r] the (shifted)
index of the child for chunk value r; a node at the last level stores ranks.
A node occupies only the slots from its first to its last occurring chunk
value; the index stored in the parent is moved back by the first value
(packing).  Children follow their parent's slots in depth-first pre-order.
This layout reproduces the worked example of the trie lookup figure; it is
used here to pin the paper's description and its memory overhead figures,
not as the GPU layout.
"""
from __future__ import annotations

import numpy as np

from ._clib import lib, ptr


def chunk_widths(M: int, R: int, short: str = "last") -> list:
    """Chunk widths least significant first.  When R does not divide M one
    chunk holds M mod R bits: the last one (short='last', as the lookup figure's
    final step t[i + alpha] implies) or the first one (short='first')."""
    n = -(-M // R)
    rem = M - (n - 1) * R
    if rem == R:
        return [R] * n
    return ([R] * (n - 1) + [rem]) if short == "last" else ([rem] + [R] * (n - 1))


def build(states, widths, full_root: bool = True, tail_pad: bool = True) -> list:
    """Packed linear trie over the sorted sector list `states` (small inputs).

    full_root keeps all 2^w0 root slots and tail_pad appends zeros so that a
    lookup of any pattern stays inside the array (safe lookup, Sec. IV)."""
    states = [int(a) for a in states]
    rank = {a: i for i, a in enumerate(states)}
    H = len(widths)
    t: list = []

    def node(members, level, B, is_root):
        w = widths[level]
        cm = (1 << w) - 1
        chunks = sorted({(a >> B) & cm for a in members})
        lo = 0 if (is_root and full_root) else chunks[0]
        hi = cm if (is_root and full_root) else chunks[-1]
        base = len(t)
        t.extend([0] * (hi - lo + 1))
        ptr_ = base - lo
        if level == H - 1:
            for a in members:
                t[ptr_ + ((a >> B) & cm)] = rank[a]
        else:
            for c in chunks:
                sub = [a for a in members if ((a >> B) & cm) == c]
                t[ptr_ + c] = node(sub, level + 1, B + w, False)
        return ptr_

    root = node(states, 0, 0, True)
    assert root == 0
    if tail_pad:
        t.extend([0] * ((1 << max(widths)) - 1))
    return t


def lookup(t, alpha: int, widths) -> int:
    """Trie lookup figure with a separate node index (reading: the loop
    variable and the node index are distinct): i <- 0; for each chunk but the
    last, i <- t[i + chunk]; the rank is t[i + last chunk]."""
    i, B = 0, 0
    for w in widths[:-1]:
        i = t[i + ((alpha >> B) & ((1 << w) - 1))]
        B += w
    return t[i + (alpha >> B)]


def packed_size(states, widths) -> int:
    """Number of slots of the packed trie with every node, root included,
    spanning [first occurring child, last occurring child] and no padding."""
    s = np.ascontiguousarray(states, dtype=np.uint64)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    n = lib().orc_trie_paper_size(ptr(s), s.size, len(widths), ptr(w))
    if n < 0:
        raise ValueError("prefix too wide for the size counter")
    return int(n)
