"""Counter-based Gaussian test matrix for step 1 of the randomized SVD.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper draws every entry of the n x r test matrix O independently from
N(0,1) (Section 2.1, step 1) but names no generator.  The reading adopted here
(so that two independent implementations, this one and the GPU one, produce
the same matrix) is:

* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4-word counter and a 2-word key; each of the ten
  rounds multiplies words 0 and 2 by the round multipliers into 2W-bit
  products and mixes the halves with words 1 and 3 and the key; the key is
  bumped by the Weyl constants between rounds.
* Key = (seed mod 2^32, floor(seed / 2^32)).  The counter of entry O[j, c]
  (0-based row j < n, column c < r) is (floor(c/4), j mod 2^32,
  floor(j / 2^32), stream), stream 0 for O.
* Uniforms u_w = (x_w + 1/2) * 2^-32, exact in FP64 and strictly in (0, 1).
* Box-Muller (1958): the pair (u0, u1) gives the entries with c = 0, 1 (mod 4)
  as rho*cos(2*pi*u1) and rho*sin(2*pi*u1), rho = sqrt(-2 ln u0); the pair
  (u2, u3) gives c = 2, 3 (mod 4) the same way.

An entry depends only on (seed, j, c): a wider sketch keeps the earlier
columns, and any row block can be generated on its own (what the block-wise
processing of Section 2.3 needs).

Parity pins (tests/test_oracle_philox.py): the generic Philox below,
instantiated with the 4x64 constants, is compared word for word with numpy's
independent Philox-4x64-10 bit generator (this pins the round structure, the
key schedule and the counter/key layout); the vectorised 4x32 form is compared
with the generic form; uniforms and Gaussians are checked statistically
(Kolmogorov-Smirnov, moments, column correlations).  No published 4x32
known-answer vector is available offline, so the 4x32 multipliers themselves
are pinned only through the 4x64 structure plus the stated constants.
"""

import numpy as np

# Round multipliers and Weyl key increments (Salmon et al., SC'11).
PHILOX_M4x32 = (0xD2511F53, 0xCD9E8D57)
PHILOX_W32 = (0x9E3779B9, 0xBB67AE85)
PHILOX_M4x64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)

STREAM_OMEGA = 0


def philox4_generic(counter, key, word_bits=32, rounds=10):
    """One Philox-4xW block on Python integers (any W); returns 4 words.

    A round maps (x0, x1, x2, x3) with key (k0, k1) to
      (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
    and the key is bumped by (W0, W1) before every round after the first.
    """
    if word_bits == 32:
        m0, m1 = PHILOX_M4x32
        w0, w1 = PHILOX_W32
    elif word_bits == 64:
        m0, m1 = PHILOX_M4x64
        w0, w1 = PHILOX_W64
    else:
        raise ValueError("word_bits must be 32 or 64")
    mask = (1 << word_bits) - 1
    x0, x1, x2, x3 = (int(v) & mask for v in counter)
    k0, k1 = (int(v) & mask for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = m0 * x0
        p1 = m1 * x2
        hi0, lo0 = p0 >> word_bits, p0 & mask
        hi1, lo1 = p1 >> word_bits, p1 & mask
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return (x0, x1, x2, x3)


def philox4x32_vec(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox-4x32 over arrays of counters (numpy uint64 lanes).

    Same rounds as philox4_generic(word_bits=32); 32x32-bit products are exact
    in uint64.  Returns four uint64 arrays holding 32-bit words.
    """
    mask = np.uint64(0xFFFFFFFF)
    sh = np.uint64(32)
    m0 = np.uint64(PHILOX_M4x32[0])
    m1 = np.uint64(PHILOX_M4x32[1])
    x0 = np.asarray(c0, dtype=np.uint64) & mask
    x1 = np.asarray(c1, dtype=np.uint64) & mask
    x2 = np.asarray(c2, dtype=np.uint64) & mask
    x3 = np.asarray(c3, dtype=np.uint64) & mask
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W32[0]) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W32[1]) & 0xFFFFFFFF
        p0 = m0 * x0
        p1 = m1 * x2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                          hi0 ^ x3 ^ np.uint64(k1), lo0)
    return x0, x1, x2, x3


def seed_key(seed):
    seed = int(seed)
    if seed < 0 or seed >= 1 << 64:
        raise ValueError("seed must be a 64-bit unsigned integer")
    return seed & 0xFFFFFFFF, seed >> 32


def raw_words(seed, rows, col_blocks, row0=0, stream=STREAM_OMEGA):
    """Raw Philox words for rows [row0, row0+rows) and column blocks
    [0, col_blocks): array of shape (rows, col_blocks, 4), dtype uint32."""
    k0, k1 = seed_key(seed)
    j = np.arange(row0, row0 + rows, dtype=np.uint64)[:, None]
    cb = np.arange(col_blocks, dtype=np.uint64)[None, :]
    x = philox4x32_vec(cb, j & np.uint64(0xFFFFFFFF), j >> np.uint64(32),
                       np.uint64(stream), k0, k1)
    return np.stack([w.astype(np.uint32) for w in x], axis=-1)


def uniforms(words):
    """u = (x + 1/2) * 2^-32 in FP64 (exact), strictly inside (0, 1)."""
    return (words.astype(np.float64) + 0.5) * (2.0 ** -32)


def box_muller(u_a, u_b):
    """Two independent N(0,1) values from two uniforms (Box & Muller, 1958)."""
    rho = np.sqrt(-2.0 * np.log(u_a))
    t = 2.0 * np.pi * u_b
    return rho * np.cos(t), rho * np.sin(t)


def gaussian_block(seed, rows, cols, row0=0, stream=STREAM_OMEGA):
    """FP64 Gaussian matrix G[j - row0, c] for j in [row0, row0+rows),
    c in [0, cols), defined entry-wise by (seed, stream, j, c)."""
    nb = (cols + 3) // 4
    w = raw_words(seed, rows, nb, row0=row0, stream=stream)
    u = uniforms(w)
    z0, z1 = box_muller(u[..., 0], u[..., 1])
    z2, z3 = box_muller(u[..., 2], u[..., 3])
    g = np.stack([z0, z1, z2, z3], axis=-1).reshape(rows, 4 * nb)
    return g[:, :cols].copy()


def omega(seed, n, r, row0=0, rows=None):
    """The n x r Gaussian test matrix O of Section 2.1, step 1 (rows
    [row0, row0+rows) of it), FP64."""
    if rows is None:
        rows = n - row0
    if row0 < 0 or rows < 0 or row0 + rows > n:
        raise ValueError("row range outside [0, n)")
    return gaussian_block(seed, rows, r, row0=row0, stream=STREAM_OMEGA)
