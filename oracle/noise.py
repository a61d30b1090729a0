"""Oracle of the noise and weight normalisation of Eq. (5) (paper Sec. III-B;
the paper's default noise is uniform on (-0.01, 0.01) at each grid point,
Sec. V-B).  TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

The noise draws its random numbers from a counter-based generator written
here from its published definition, Philox4x32-10 (Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011): the state is
a 128-bit counter (four 32-bit words) and a 64-bit key; each of ten rounds
multiplies words 0 and 2 by two fixed 32-bit constants, exchanges the high
and low halves of the 64-bit products with the other words XORed with the
key, and advances the key by two Weyl constants.  Counter = (cell low, cell
high, field low, field high), key = (seed low, seed high).  Plain numpy with
uint64 arithmetic, vectorised over the counters.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit words (held in uint64).
    Returns the four output words as uint64 arrays."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for _ in range(10):
        p0 = _M0 * c0  # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def _bits52(hi, lo):
    return (hi << np.uint64(20)) | (lo >> np.uint64(12))


def noise(n: int, m: int, kind: int, amplitude: float, seed: int, field_offset: int = 0) -> np.ndarray:
    """E (m, n): the noise of fields field_offset .. field_offset + m - 1 at
    cells 0 .. n - 1.  kind 1: uniform amplitude ((2u + 1) 2^-52 - 1) with u
    the 52 bits of output words 0-1 (on (-amplitude, amplitude), exact
    before the product); kind 2: Gaussian by Box-Muller, amplitude
    sqrt(-2 ln x1) cos(2 pi x2) with x = (u + 1/2) 2^-52 from words 0-1 and
    2-3; kind 0: zeros."""
    if kind == 0:
        return np.zeros((m, n))
    cells = np.arange(n, dtype=np.uint64)
    fields = np.uint64(field_offset) + np.arange(m, dtype=np.uint64)
    C0 = np.broadcast_to(cells[None, :] & _MASK, (m, n))
    C1 = np.broadcast_to(cells[None, :] >> _S32, (m, n))
    C2 = np.broadcast_to((fields & _MASK)[:, None], (m, n))
    C3 = np.broadcast_to((fields >> _S32)[:, None], (m, n))
    seed = np.uint64(seed)
    r0, r1, r2, r3 = philox4x32_10(C0, C1, C2, C3, seed & _MASK, seed >> _S32)
    u = _bits52(r0, r1)
    if kind == 1:
        return amplitude * ((2.0 * u.astype(np.float64) + 1.0) * 2.0 ** -52 - 1.0)
    x1 = (u.astype(np.float64) + 0.5) * 2.0 ** -52
    x2 = (_bits52(r2, r3).astype(np.float64) + 0.5) * 2.0 ** -52
    return amplitude * (np.sqrt(-2.0 * np.log(x1)) * np.cos(2.0 * np.pi * x2))


def normalize_weights(mu: np.ndarray, min_abs_sum: float):
    """alpha_i = mu_i / sum_j mu_j per field (Eq. (5)); mu (m, s), the sum in
    index order.  Fields with |sum| < min_abs_sum keep mu and are flagged.
    Returns (alpha, flags)."""
    mu = np.asarray(mu, dtype=np.float64)
    alpha = mu.copy()
    flags = np.zeros(mu.shape[0], dtype=np.int32)
    for j in range(mu.shape[0]):
        sm = 0.0
        for k in range(mu.shape[1]):
            sm += mu[j, k]
        if not abs(sm) >= min_abs_sum:
            flags[j] = 1
            continue
        alpha[j] = mu[j] / sm
    return alpha, flags
