"""Counter-based random numbers for the noisy densification (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper regenerates the background of a densified frame "with noise" for
programs that analyse the noise level (Sec. 3.2) but fixes no generator.  The
reading used on both sides is a counter-based generator, so that every pixel
of every frame draws the same numbers whatever the batch or launch shape:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key pass
  through ten rounds; each round multiplies counter words 0 and 2 by fixed
  32-bit constants, keeps both halves of the 64-bit products and mixes the
  high halves with the other two words and the round key; the key advances by
  two Weyl constants between rounds.  Written here from that definition and
  checked against the published known-answer vectors of the generator.
* Uniforms from 32-bit words w: u1 = (floor(w / 2^8) + 1) 2^-24 in (0, 1] and
  u2 = floor(w / 2^8) 2^-24 in [0, 1) -- 24-bit values, exact in float32.
* Normals by the Box-Muller transform (Box and Muller, 1958):
  r = sqrt(-2 ln u1), z_a = r cos(2 pi u2), z_b = r sin(2 pi u2), two
  independent standard normals per pair of uniforms.

These are plain Python-integer / NumPy uint64 computations in the order the
definitions state them, vectorised over counters.
"""

from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57      # round multipliers of Philox4x32
W0, W1 = 0x9E3779B9, 0xBB67AE85      # key increments (golden ratio, sqrt(3) - 1)
ROUNDS = 10
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key, rounds=ROUNDS):
    """Philox4x32-R of counters [..., 4] (uint32 values) under key (k0, k1).

    Returns uint64 arrays [..., 4] holding the four 32-bit output words.
    """
    c = [np.asarray(counter, dtype=np.uint64)[..., j] & _MASK for j in range(4)]
    k0, k1 = np.uint64(key[0]) & _MASK, np.uint64(key[1]) & _MASK
    for r in range(rounds):
        p0 = np.uint64(M0) * c[0]          # < 2^64: 32 x 32-bit product
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return np.stack(c, axis=-1)


def uniform_open0(w):
    """u in (0, 1] from 32-bit words: (top 24 bits + 1) / 2^24."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 1.0) * 2.0 ** -24


def uniform_open1(w):
    """u in [0, 1) from 32-bit words: top 24 bits / 2^24."""
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def box_muller(u1, u2):
    """Two standard normals (z_a, z_b) from u1 in (0, 1], u2 in [0, 1)."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def seed_key(seed):
    """Philox key of a 64-bit seed: (low word, high word)."""
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return s & 0xFFFFFFFF, s >> 32


def pixel_normals(seed, frame, n_pix):
    """(z_a, z_b) of every pixel of one frame, float64 [n_pix] each.

    Pixel i uses block g = i // 2 of counter (g, frame, 0, 0) under the seed's
    key; the even pixel of the block takes words (0, 1) as (u1, u2), the odd
    pixel words (2, 3).
    """
    n_blk = (n_pix + 1) // 2
    ctr = np.zeros((n_blk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n_blk, dtype=np.uint64)
    ctr[:, 1] = np.uint64(int(frame) & 0xFFFFFFFF)
    w = philox4x32(ctr, seed_key(seed))
    w1 = w[:, [0, 2]].reshape(-1)[:n_pix]
    w2 = w[:, [1, 3]].reshape(-1)[:n_pix]
    return box_muller(uniform_open0(w1), uniform_open1(w2))


def truncated(za, zb, t):
    """The pixel's draw, at most t: z_a if z_a <= t, else z_b if z_b <= t, else t."""
    return np.where(za <= t, za, np.where(zb <= t, zb, t))
