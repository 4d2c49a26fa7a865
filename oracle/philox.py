"""Philox4x32-10 and the SSQA random-bit stream.  Test infrastructure (see package doc).

Generator: Philox4x32 with 10 rounds, from J. K. Salmon, M. A. Moraes,
R. O. Dror and D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11.  A 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1) go through
ten rounds.  Each round multiplies c0 and c2 by the two Philox multipliers,
keeping the high and low 32-bit halves, and mixes them with c1, c3 and the key;
between rounds the key is advanced by the two Weyl increments.

Stream layout used by the annealer (both the oracle and the HIP library follow
it, each with its own code):

* key    = (low 32 bits of seed, high 32 bits of seed)
* counter = (tag, i >> 7, k, b): tag 0 draws the initial spins, tag t+1 draws the
  noise r(t) of the update t -> t+1; i is the spin, k the replica, b the trial.
* spin i takes bit (i & 31) of output word (i & 127) >> 5; bit 1 means +1.

The noise r_{i,k}(t) is therefore independent per spin, replica, cycle and
trial (Eq. 6a writes r_i(t) without a replica index; the per-replica reading is
the one under which the replicas search independently, Section 3.2).
"""

from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Round multipliers and key increments published with Philox4x32.
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs are integer arrays (broadcastable) holding
    32-bit values; returns four uint64 arrays holding the 32-bit output words."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0          # < 2**64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def seed_key(seed: int) -> tuple[int, int]:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def stream_bits(seed: int, tag: int, n_spins: int, replicas, trials) -> np.ndarray:
    """Random bits of one tag for every (trial b, replica k, spin i).

    ``replicas`` and ``trials`` are index sequences (or counts).  Returns uint8
    [len(trials), len(replicas), n_spins] with entries 0/1.
    """
    ks = np.arange(replicas) if np.isscalar(replicas) else np.asarray(replicas)
    bs = np.arange(trials) if np.isscalar(trials) else np.asarray(trials)
    k0, k1 = seed_key(seed)
    groups = (n_spins + 127) // 128
    g = np.arange(groups, dtype=np.uint64)
    # counter (tag, group, k, b); broadcast to [B, K, G]
    B = bs.astype(np.uint64)[:, None, None]
    K = ks.astype(np.uint64)[None, :, None]
    G = g[None, None, :]
    words = philox4x32_10(np.uint64(tag), G, K, B, k0, k1)
    w = np.stack(words, axis=-1)                        # [B, K, G, 4]
    i = np.arange(n_spins)
    word = w[:, :, i >> 7, (i & 127) >> 5]              # [B, K, N]
    bits = (word >> (i & 31).astype(np.uint64)) & np.uint64(1)
    return bits.astype(np.uint8)


def stream_signs(seed: int, tag: int, n_spins: int, replicas, trials) -> np.ndarray:
    """The same bits as +-1 (int64): bit 1 -> +1, bit 0 -> -1."""
    return 2 * stream_bits(seed, tag, n_spins, replicas, trials).astype(np.int64) - 1
