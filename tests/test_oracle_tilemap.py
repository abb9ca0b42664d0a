"""Pins of the block-cyclic tile maps (Sections 2.3 and 3.1) by brute force."""
import numpy as np
import pytest

from oracle import tilemap as T


@pytest.mark.parametrize("N,b,P", [(1, 1, 1), (10, 3, 1), (10, 3, 2), (17, 4, 3), (100, 7, 4),
                                   (50000, 4096, 1), (20000, 4096, 3)])
def test_block_cyclic_map_is_a_bijection(N, b, P):
    seen = {}
    for g in range(N):
        t = g // b
        key = (T.owner(t, P), T.local_offset(g, b, P))
        assert key not in seen
        seen[key] = g
    counts = [T.numroc(N, b, p, P) for p in range(P)]
    assert sum(counts) == N
    for p in range(P):
        offs = sorted(off for (o, off) in seen if o == p)
        assert offs == list(range(counts[p]))      # dense local storage


def test_tiles_cover_without_padding():
    for N, b in [(848, 4096), (50000, 4096), (20000, 4096), (200000, 8192), (100000, 8192)]:
        nt = T.num_tiles(N, b)
        spans = [T.tile_range(t, N, b) for t in range(nt)]
        assert spans[0][0] == 0 and spans[-1][1] == N
        assert all(spans[i][1] == spans[i + 1][0] for i in range(nt - 1))


def test_workload_edge_tiles():
    # dense workloads: 50000 x 20000 in 4096 tiles, 200000 x 100000 in 8192 tiles
    d = T.tile_descriptors(50000, 20000, 4096, 4096)
    assert len(d) == 13 * 5
    assert d[-1, 3] == 848 and d[-1, 5] == 3616
    d = T.tile_descriptors(200000, 100000, 8192, 8192)
    assert len(d) == 25 * 13
    assert d[-1, 3] == 3392 and d[-1, 5] == 1696


def test_visit_orders_are_permutations_and_serpentine():
    TI, TJ = 4, 3
    prev_last = None
    for t in range(6):
        v = T.visit_order(TI, TJ, t)
        assert sorted(v.tolist()) == list(range(TI * TJ))
        if prev_last is not None:
            assert v[0] == prev_last
        prev_last = v[-1]


def test_csr_row_blocks_skip_empty():
    rowptr = np.array([0, 2, 2, 2, 2, 5, 5, 6])
    blocks = T.row_blocks(rowptr, 2)
    assert blocks.tolist() == [[0, 2, 0, 2], [4, 2, 2, 5], [6, 1, 5, 6]]


def test_blockwise_product_equals_plain_product():
    # Section 2.3, Eq. (3): the block-wise product is the plain product, with
    # the same number of scalar multiplications
    rng = np.random.default_rng(0)
    X = rng.standard_normal((37, 23))
    Y = rng.standard_normal((23, 11))
    b = 8
    out = np.zeros((37, 11))
    mults = 0
    for I in range(T.num_tiles(37, b)):
        r0, r1 = T.tile_range(I, 37, b)
        for J in range(T.num_tiles(23, b)):
            c0, c1 = T.tile_range(J, 23, b)
            out[r0:r1] += X[r0:r1, c0:c1] @ Y[c0:c1]
            mults += (r1 - r0) * (c1 - c0) * 11
    assert mults == 37 * 23 * 11
    assert np.allclose(out, X @ Y, rtol=1e-13, atol=1e-13)
