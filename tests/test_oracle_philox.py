"""Pins of the oracle's counter-based Gaussian generator (Section 2.1, step 1)."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as P


def test_generic_philox4x64_matches_numpy_bit_generator():
    # numpy's Philox is an independent Philox-4x64-10; it increments the
    # counter before each block, so block b uses counter (start + b + 1).
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr = [int(x) for x in rng.integers(0, 2**62, size=4, dtype=np.int64)]
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array(ctr, dtype=np.uint64))
        raw = [int(x) for x in bg.random_raw(12)]
        for b in range(3):
            c = list(ctr)
            c[0] += b + 1
            assert list(P.philox4_generic(c, key, 64)) == raw[4 * b:4 * b + 4]


def test_weyl_constants_are_the_64bit_ones_truncated():
    assert P.PHILOX_W32[0] == P.PHILOX_W64[0] >> 32
    assert P.PHILOX_W32[1] == P.PHILOX_W64[1] >> 32


def test_vectorised_4x32_equals_generic():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**32, size=(4, 64), dtype=np.uint64)
    for key in [(0, 0), (123456789, 987654321), (2**32 - 1, 2**32 - 1)]:
        v = P.philox4x32_vec(c[0], c[1], c[2], c[3], key[0], key[1])
        for i in range(c.shape[1]):
            g = P.philox4_generic([int(c[w, i]) for w in range(4)], key, 32)
            assert tuple(int(v[w][i]) for w in range(4)) == g


def test_round_count_matters():
    a = P.philox4_generic((1, 2, 3, 4), (5, 6), 32, rounds=10)
    b = P.philox4_generic((1, 2, 3, 4), (5, 6), 32, rounds=9)
    assert a != b


def test_uniforms_strictly_inside_unit_interval():
    w = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32)
    u = P.uniforms(w)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 0.5 * 2.0**-32 and u[-1] == 1.0 - 0.5 * 2.0**-32


def test_raw_words_uniform_statistics():
    w = P.raw_words(seed=11, rows=4096, col_blocks=8)
    u = P.uniforms(w).ravel()
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # every bit position is fair
    bits = ((w.ravel()[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def test_omega_gaussian_statistics():
    O = P.omega(seed=0, n=8192, r=64)
    z = O.ravel()
    assert np.all(np.isfinite(z))
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 6.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    C = np.corrcoef(O.T)
    off = C[~np.eye(64, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(O.shape[0])
    # the four outputs of one block (same row, columns 4b..4b+3) are independent too
    for c in range(1, 4):
        assert abs(np.corrcoef(O[:, 0], O[:, c])[0, 1]) < 5.0 / np.sqrt(O.shape[0])


def test_omega_entrywise_definition_properties():
    full = P.omega(seed=42, n=300, r=13)
    # any row block can be generated on its own
    assert np.array_equal(P.omega(seed=42, n=300, r=13, row0=37, rows=100), full[37:137])
    # a wider sketch keeps the earlier columns
    assert np.array_equal(P.omega(seed=42, n=300, r=20)[:, :13], full)
    # different seeds and streams give different matrices
    assert not np.array_equal(P.omega(seed=43, n=300, r=13), full)
    other = P.gaussian_block(42, 300, 13, stream=1)
    assert not np.array_equal(other, full)


def test_seed_key_split():
    assert P.seed_key(0) == (0, 0)
    assert P.seed_key(2**32 + 5) == (5, 1)
    with pytest.raises(ValueError):
        P.seed_key(-1)
