"""Philox4x32-10 counter-based generator and the Gaussian map used by every sketch.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The paper draws its randomized-SVD sketches from a Gaussian distribution but does not
fix a generator (randomized SVD with q QR iterations, Introduction and Table 1).  Both
the oracle and the GPU path therefore implement one published counter-based generator,
Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), each from that definition and independently of the other.

Philox4x32 round (from the SC'11 paper): with the two 32x32->64 multipliers M0, M1,
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2
    c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
and the key is advanced by the Weyl constants (W0, W1) between rounds.

Gaussian map (a reading of this implementation, not the paper's): element e of a
sketch drawn at RG step `step` for call-site `site` uses the counter
(lo32(e>>1), hi32(e>>1), step, site) and key (lo32(seed), hi32(seed)).  The four output
words give two 53-bit uniforms
    u1 = ((x0>>5)*2^26 + (x1>>6) + 1) * 2^-53   in (0, 1]
    u2 = ((x2>>5)*2^26 + (x3>>6))     * 2^-53   in [0, 1)
and Box-Muller gives r*cos(2 pi u2) for even e and r*sin(2 pi u2) for odd e, with
r = sqrt(-2 ln u1).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_THREADS = max(1, min(16, os.cpu_count() or 1))

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """Apply Philox4x32-10.

    ctr: uint64 array of shape (4, n) holding 32-bit words; key: uint64 array (2, n) or (2,).
    Returns a uint64 array (4, n) of 32-bit output words.
    """
    c0, c1, c2, c3 = (np.asarray(w, dtype=np.uint64) & _MASK for w in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # < 2^64: product of two 32-bit numbers
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return np.stack([c0, c1, c2, c3])


def gaussian(seed, step, site, n, offset=0):
    """n standard normals for elements offset .. offset+n-1 (float64)."""
    p_lo = offset >> 1
    p_hi = (offset + n + 1) >> 1
    pairs = np.empty((p_hi - p_lo, 2))
    chunk = 1 << 17          # work in cache-sized pieces; the values do not depend on it
    bounds = [(lo, min(p_hi, lo + chunk)) for lo in range(p_lo, p_hi, chunk)]

    def work(b):
        pairs[b[0] - p_lo:b[1] - p_lo] = _gaussian_pairs(seed, step, site, b[0], b[1])

    with ThreadPoolExecutor(max_workers=_THREADS) as ex:
        list(ex.map(work, bounds))
    flat = pairs.reshape(-1)
    start = offset - 2 * p_lo
    return flat[start:start + n].copy()


def _gaussian_pairs(seed, step, site, p_lo, p_hi):
    """Both Box-Muller outputs (cos, sin) for counter pairs p_lo .. p_hi-1."""
    return _gaussian_pairs_at(seed, step, site, np.arange(p_lo, p_hi, dtype=np.uint64))


def _gaussian_pairs_at(seed, step, site, pair):
    """Both Box-Muller outputs (cos, sin) for an array of counter pairs."""
    zeros = np.zeros_like(pair)
    ctr = (pair & _MASK, pair >> np.uint64(32), zeros + np.uint64(step), zeros + np.uint64(site))
    seed = int(seed)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    x = philox4x32_10(ctr, key)
    two26 = 67108864.0
    scale = 2.0 ** -53
    u1 = ((x[0] >> np.uint64(5)).astype(np.float64) * two26
          + (x[1] >> np.uint64(6)).astype(np.float64) + 1.0) * scale
    u2 = ((x[2] >> np.uint64(5)).astype(np.float64) * two26
          + (x[3] >> np.uint64(6)).astype(np.float64)) * scale
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    return np.stack([r * np.cos(theta), r * np.sin(theta)], axis=1)


def gaussian_at(seed, step, site, e):
    """Standard normals for an arbitrary array of element numbers e (uint64)."""
    e = np.asarray(e, dtype=np.uint64).reshape(-1)
    out = np.empty(e.size)
    chunk = 1 << 17

    def work(lo):
        ee = e[lo:lo + chunk]
        pr = _gaussian_pairs_at(seed, step, site, ee >> np.uint64(1))
        odd = (ee & np.uint64(1)).astype(bool)
        out[lo:lo + chunk] = np.where(odd, pr[:, 1], pr[:, 0])

    with ThreadPoolExecutor(max_workers=_THREADS) as ex:
        list(ex.map(work, range(0, e.size, chunk)))
    return out


def gaussian_matrix_t(seed, step, site, rows, cols):
    """Transpose (cols x rows) of gaussian_matrix(seed, step, site, rows, cols)."""
    j = np.arange(cols, dtype=np.uint64)[:, None]
    i = np.arange(rows, dtype=np.uint64)[None, :]
    return gaussian_at(seed, step, site, i * np.uint64(cols) + j).reshape(cols, rows)


def gaussian_matrix(seed, step, site, rows, cols):
    """Row-major rows x cols sketch: element (i, j) is element number i*cols + j."""
    return gaussian(seed, step, site, rows * cols).reshape(rows, cols)
