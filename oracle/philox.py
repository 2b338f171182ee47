"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) and the collocation
point sampler built on it (oracle side, numpy).

Round: (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
lo(M0 c0)) with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by
(0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.

Sampling (paper Sec. 3: residuals on randomly sampled points): interior point i
of step s uses counter (i, s_lo, s_hi, 0), boundary point b uses
(b, s_lo, s_hi, 1), key = (seed_lo, seed_hi).  Coordinates are integers on the
2^-22 lattice drawn by the multiply-shift range reduction j = (r * M) >> 32.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr[..., 4] uint32, key[..., 2] uint32 -> uint32[..., 4]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32)
    k1 = np.asarray(key[..., 1], dtype=np.uint32)
    with np.errstate(over="ignore"):
        for r in range(10):
            p0 = c[0].astype(np.uint64) * M0
            p1 = c[2].astype(np.uint64) * M1
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            if r < 9:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
    return np.stack(c, axis=-1)


LATTICE = 1 << 22


def _range(r, m):
    return ((r.astype(np.uint64) * np.uint64(m)) >> np.uint64(32)).astype(np.int64)


def sample_points(d: int, h: float, n: int, nb: int, seed: int, step: int):
    """Interior points on the lattice in [-1+h, 1-h]^d and boundary points on
    the faces of [-1,1]^d, as float64 arrays (exact lattice values)."""
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    slo, shi = step & 0xFFFFFFFF, (step >> 32) & 0xFFFFFFFF
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint64).astype(np.uint32)
    ctr[:, 1], ctr[:, 2], ctr[:, 3] = slo, shi, 0
    r = philox4x32_10(ctr, np.broadcast_to(key, (n, 2)))
    jh = int(round(h * LATTICE))
    m_int = 2 * LATTICE - 2 * jh + 1
    pts = np.empty((n, d))
    for a in range(d):
        pts[:, a] = (_range(r[:, a], m_int) + (jh - LATTICE)) / LATTICE
    ctr = np.zeros((nb, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(nb, dtype=np.uint64).astype(np.uint32)
    ctr[:, 1], ctr[:, 2], ctr[:, 3] = slo, shi, 1
    r = philox4x32_10(ctr, np.broadcast_to(key, (nb, 2)))
    m_b = 2 * LATTICE + 1
    bpts = np.empty((nb, d))
    for a in range(d):
        bpts[:, a] = (_range(r[:, a], m_b) - LATTICE) / LATTICE
    face = _range(r[:, 3], 2 * d)
    bpts[np.arange(nb), face // 2] = np.where(face % 2 == 0, -1.0, 1.0)
    return pts, bpts
