"""Integer bookkeeping of the TLR factorization (oracle O8).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

These are the integer arrays the GPU library must reproduce bit for bit:
tile offsets in the factor arenas, the widths of the block-row panels, the
order in which "sortRanks" presents the tiles of a column (Section 4.2), and
the evolution of the active subset under "getConvergedTiles" /
"updateSubset" (Algorithm "Left Looking Cholesky TLR ARA Update").
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def lower_offsets(ranks: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum of the ranks of the strictly lower tiles, taken in
    row-major lower order ((1,0), (2,0), (2,1), (3,0), ...).

    Element (i, j), i > j, is the first column of tile (i, j) in an arena
    that stores all U (or all V) factors side by side; -1 elsewhere.  The
    last entry returned separately is the arena width.
    """
    nb = ranks.shape[0]
    off = np.full((nb, nb), -1, dtype=np.int64)
    acc = 0
    for i in range(nb):
        for j in range(i):
            off[i, j] = acc
            acc += int(ranks[i, j])
    return off, acc


def row_panel_offsets(ranks: np.ndarray) -> np.ndarray:
    """Column of tile (i, j) inside block row i's panel [L_i0 | L_i1 | ...]:
    sum_{j' < j} r_ij'.  -1 on and above the diagonal."""
    nb = ranks.shape[0]
    off = np.full((nb, nb), -1, dtype=np.int64)
    for i in range(nb):
        acc = 0
        for j in range(i):
            off[i, j] = acc
            acc += int(ranks[i, j])
    return off


def row_widths(ranks: np.ndarray, k: int) -> np.ndarray:
    """R_i^(k) = sum_{j<k} r_ij for every block row i: the width of row i's
    panel when column k is processed."""
    nb = ranks.shape[0]
    return np.array([int(ranks[i, :min(k, i)].sum()) for i in range(nb)], dtype=np.int64)


def sort_ranks(a_ranks: np.ndarray, k: int) -> List[int]:
    """"sortRanks": the rows i > k of column k ordered by the input rank a_ik,
    descending, ties broken by ascending i (Section 4.2)."""
    nb = a_ranks.shape[0]
    rows = list(range(k + 1, nb))
    return sorted(rows, key=lambda i: (-int(a_ranks[i, k]), i))


def active_sets(order: Sequence[int], s_max: int, flags: Sequence[Sequence[bool]]) -> List[List[int]]:
    """Evolution of the active subset of one column.

    The first subset is the first s_max tiles of the sorted order.  After an
    iteration, `flags[t][p]` tells whether the tile at position p of the
    current subset converged.  "updateSubset" keeps the unconverged tiles in
    their order and appends, in sorted order, as many of the not yet started
    tiles as converged, so the subset never exceeds s_max.  Returns the
    subsets seen by the successive iterations (ending with the empty one, if
    the flags reach it).
    """
    active = list(order[:s_max])
    waiting = list(order[s_max:])
    out = [list(active)]
    for f in flags:
        if len(f) != len(active):
            raise ValueError("flag vector length %d != subset size %d" % (len(f), len(active)))
        keep = [t for t, c in zip(active, f) if not c]
        refill = len(active) - len(keep)
        active = keep + waiting[:refill]
        waiting = waiting[refill:]
        out.append(list(active))
        if not active:
            break
    return out


def tile_rows(n: int, m: int) -> np.ndarray:
    """Number of real (unpadded) rows of every block row."""
    nb = -(-n // m)
    return np.array([min(m, n - k * m) for k in range(nb)], dtype=np.int64)
