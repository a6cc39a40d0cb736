"""Counter-based Gaussian sketch for the oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything under ``oracle/``.

The paper only asks for Pi ~ N(0,1)^{d x k} (Algorithm 2, step 1).  Both the
oracle and the GPU library draw it from a seed with Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), each
from that published definition, with this mapping to normals:

* Pi is d x k row-major; element e = r*k + c.  Normals 2j and 2j+1 come from
  one Philox call with counter (j mod 2^32, j div 2^32, 0, 0) and key
  (seed mod 2^32, seed div 2^32), giving words x0..x3.
* u1 = ((x0 >> 5) * 2^26 + (x1 >> 6) + 1) * 2^-53  in (0, 1],
  u2 = ((x2 >> 5) * 2^26 + (x3 >> 6)) * 2^-53      in [0, 1).
* Box-Muller in float64: rho = sqrt(-2 ln u1),
  z_2j = rho cos(2 pi u2), z_2j+1 = rho sin(2 pi u2).

The Philox words are pinned bit for bit by published known-answer vectors;
the Box-Muller normals are pinned by their distribution (moments, KS test).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.

    ``ctr``: array (..., 4) of uint32 counters; ``key``: (2,) uint32.
    Returns an array (..., 4) of uint32 words."""
    c = np.asarray(ctr, dtype=np.uint64)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # 32 x 32 -> 64 bit products fit in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_words(seed: int, pairs: int) -> np.ndarray:
    """Words for pair indices j = 0..pairs-1 (shape (pairs, 4), uint32)."""
    j = np.arange(pairs, dtype=np.uint64)
    ctr = np.zeros((pairs, 4), dtype=np.uint64)
    ctr[:, 0] = j & _MASK
    ctr[:, 1] = j >> _S32
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return philox4x32_10(ctr, key)


def gaussian(seed: int, rows: int, cols: int) -> np.ndarray:
    """The rows x cols N(0,1) sketch in float64 (row-major element order)."""
    total = rows * cols
    pairs = (total + 1) // 2
    w = philox_words(seed, pairs).astype(np.uint64)
    two53 = 2.0 ** -53
    a = (w[:, 0] >> np.uint64(5)).astype(np.float64) * 67108864.0
    u1 = (a + (w[:, 1] >> np.uint64(6)).astype(np.float64) + 1.0) * two53
    b = (w[:, 2] >> np.uint64(5)).astype(np.float64) * 67108864.0
    u2 = (b + (w[:, 3] >> np.uint64(6)).astype(np.float64)) * two53
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = 6.283185307179586 * u2
    z = np.empty(2 * pairs)
    z[0::2] = rho * np.cos(ang)
    z[1::2] = rho * np.sin(ang)
    return z[:total].reshape(rows, cols)
