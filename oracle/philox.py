"""Counter-based Gaussian perturbations.  Test infrastructure only.

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a
2x32-bit key pass through ten rounds; each round multiplies counter words 0
and 2 by two fixed odd constants, keeps the 64-bit products' halves and mixes
the high halves with the other counter words and the round key; the key is
bumped by two Weyl constants between rounds.

Normals come from the Box-Muller transform.  The mapping from (seed, stream,
row, column) to counters and bits is the one the device sampler documents
in its C header; this file writes it out independently so that the device
output can be checked element by element.

Mapping (n x K matrix W, sample index fastest, K_draw = K/2 when antithetic):
  counter = (column s, row block b, stream_lo, stream_hi), key = (seed_lo, seed_hi)
  FP32: block b covers rows 4b..4b+3; words (x0, x1) -> rows 4b, 4b+1 and
        (x2, x3) -> rows 4b+2, 4b+3 with u1 = ((x>>8)+1) 2^-24, u2 = (x>>8) 2^-24.
  FP64: block b covers rows 2b, 2b+1; u1 = (((x0<<21)|(x1>>11))+1) 2^-53,
        u2 = ((x2<<21)|(x3>>11)) 2^-53.
  z_a = sqrt(-2 ln u1) cos(2 pi u2),  z_b = sqrt(-2 ln u1) sin(2 pi u2).
  W[i, s] = sigma z, and with antithetic pairs W[i, s + K/2] = -W[i, s].
"""
from __future__ import annotations

import numpy as np

_MUL0 = 0xD2511F53
_MUL1 = 0xCD9E8D57
_WEYL0 = 0x9E3779B9
_WEYL1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def _mulhilo(a, b):
    p = np.asarray(a, dtype=np.uint64) * np.uint64(b)
    return (p >> np.uint64(32)).astype(np.uint64), (p & np.uint64(_MASK)).astype(np.uint64)


def philox4x32_10(counter, key):
    """counter: 4 arrays (broadcastable) of uint32 words; key: 2 words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(_MASK) for c in counter)
    k0 = np.uint64(int(key[0]) & _MASK)
    k1 = np.uint64(int(key[1]) & _MASK)
    for rnd in range(10):
        if rnd:
            k0 = np.uint64((int(k0) + _WEYL0) & _MASK)
            k1 = np.uint64((int(k1) + _WEYL1) & _MASK)
        hi0, lo0 = _mulhilo(c0, _MUL0)
        hi1, lo1 = _mulhilo(c2, _MUL1)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def _box_muller(u1, u2):
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    return rad * np.cos(th), rad * np.sin(th)


def normals(n: int, K_draw: int, seed: int, stream: int, dtype: str):
    """Standard normals Z (n, K_draw) in float64 following the mapping above."""
    s = np.arange(K_draw, dtype=np.uint64)[None, :]
    key = (seed & _MASK, (seed >> 32) & _MASK)
    st_lo, st_hi = stream & _MASK, (stream >> 32) & _MASK
    if dtype == "f32":
        nb = (n + 3) // 4
        b = np.arange(nb, dtype=np.uint64)[:, None]
        x0, x1, x2, x3 = philox4x32_10((s + 0 * b, b + 0 * s, st_lo, st_hi), key)
        f = lambda x: (x.astype(np.float64) // 256)  # noqa: E731  (x >> 8)
        za, zb = _box_muller((f(x0) + 1.0) * 2.0 ** -24, f(x1) * 2.0 ** -24)
        zc, zd = _box_muller((f(x2) + 1.0) * 2.0 ** -24, f(x3) * 2.0 ** -24)
        Z = np.stack([za, zb, zc, zd], axis=1).reshape(4 * nb, K_draw)
    elif dtype == "f64":
        nb = (n + 1) // 2
        b = np.arange(nb, dtype=np.uint64)[:, None]
        x0, x1, x2, x3 = philox4x32_10((s + 0 * b, b + 0 * s, st_lo, st_hi), key)
        w = lambda hi, lo: ((hi.astype(np.uint64) << np.uint64(21)) | (lo.astype(np.uint64) >> np.uint64(11)))  # noqa: E731
        u1 = (w(x0, x1).astype(np.float64) + 1.0) * 2.0 ** -53
        u2 = w(x2, x3).astype(np.float64) * 2.0 ** -53
        za, zb = _box_muller(u1, u2)
        Z = np.stack([za, zb], axis=1).reshape(2 * nb, K_draw)
    else:
        raise ValueError(dtype)
    return Z[:n]


def perturbations(n: int, K: int, sigma: float, seed: int, stream: int,
                  dtype: str, antithetic: bool = True):
    """W (n, K) as the device sampler defines it."""
    if antithetic:
        Z = normals(n, K // 2, seed, stream, dtype)
        return sigma * np.concatenate([Z, -Z], axis=1)
    return sigma * normals(n, K, seed, stream, dtype)
