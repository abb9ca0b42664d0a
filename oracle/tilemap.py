"""Block-cyclic tile maps and pass visit orders (Sections 2.3 and 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1: every operation works on blocks that are ranges of row and column
indices of the source matrix, their number set by the memory limits; Section
2.3 (Eq. (3)) shows that a product computed block by block equals the plain
product with the same operation count, and the introduction ties the layout
to ScaLAPACK's block-cyclic distribution.  The oracle spells the layout out
with ScaLAPACK's conventions (0-based, first block on process 0):

* N indices in blocks of b: tile t covers [t*b, min((t+1)*b, N)); the last
  tile may be partial, there is no padding.
* On a 1-D grid of P processes: owner(t) = t mod P, local tile = t div P,
  local offset of global index g = ((g div b) div P)*b + g mod b, and the
  number of indices process p holds is
  (N div (b P))*b + min(max(N mod (b P) - p b, 0), b).
* A 2-D grid P x Q is the product of a row grid and a column grid.
* Visit orders of the passes over A (passes numbered 0 .. 2q+1): the sketch
  and every A-product (even passes) go row-major over (I, J) forward; every
  A^T-product (odd passes) goes column-major backward, so each pass starts on
  the tile where the previous one ended.

Parity pins (tests/test_oracle_tilemap.py): brute-force enumeration of every
global index (the map is a bijection onto (owner, local offset)), per-process
counts sum to N, and the edge sizes of the two dense block-cyclic workloads
(50000 x 20000 in 4096 tiles: 848 and 3616; 200000 x 100000 in 8192 tiles:
3392 and 1696).
"""

import numpy as np


def num_tiles(N, b):
    if N < 0 or b < 1:
        raise ValueError("need N >= 0, b >= 1")
    return (N + b - 1) // b


def tile_range(t, N, b):
    lo = t * b
    return lo, min(lo + b, N)


def owner(t, P):
    return t % P


def local_tile(t, P):
    return t // P


def local_offset(g, b, P):
    return ((g // b) // P) * b + g % b


def numroc(N, b, p, P):
    """Number of the N indices that process p of P holds."""
    return (N // (b * P)) * b + min(max(N % (b * P) - p * b, 0), b)


def tile_descriptors(m, n, bm, bn, P=1, Q=1):
    """One row per tile in I-major order:
    (I, J, row0, rows, col0, cols, owner_p, owner_q, local_I, local_J,
     local_row0, local_col0), int64."""
    TI, TJ = num_tiles(m, bm), num_tiles(n, bn)
    rows = []
    for I in range(TI):
        r0, r1 = tile_range(I, m, bm)
        for J in range(TJ):
            c0, c1 = tile_range(J, n, bn)
            rows.append((I, J, r0, r1 - r0, c0, c1 - c0,
                         owner(I, P), owner(J, Q), local_tile(I, P), local_tile(J, Q),
                         local_offset(r0, bm, P), local_offset(c0, bn, Q)))
    return np.array(rows, dtype=np.int64).reshape(-1, 12)


def visit_order(TI, TJ, pass_index):
    """Linear tile indices (I*TJ + J) in the order pass `pass_index` visits
    them: even passes row-major forward, odd passes column-major backward."""
    if pass_index % 2 == 0:
        return np.array([I * TJ + J for I in range(TI) for J in range(TJ)], dtype=np.int64)
    return np.array([I * TJ + J for J in range(TJ - 1, -1, -1) for I in range(TI - 1, -1, -1)],
                    dtype=np.int64)


def row_blocks(rowptr, br):
    """Row blocks of a CSR matrix: (row0, rows, nnz_begin, nnz_end) for each
    block of br rows, empty blocks (no stored entries) dropped (Section 3.1:
    blocks that hold no values are skipped)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    m = len(rowptr) - 1
    out = []
    for r0 in range(0, m, br):
        r1 = min(m, r0 + br)
        a, b = int(rowptr[r0]), int(rowptr[r1])
        if b > a:
            out.append((r0, r1 - r0, a, b))
    return np.array(out, dtype=np.int64).reshape(-1, 4)
