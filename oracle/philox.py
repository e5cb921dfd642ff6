"""Philox4x32-10 counter-based generator, NumPy version (test infrastructure only).

Written from the published description (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a
2-word key; each of the 10 rounds multiplies words 0 and 2 by the two Philox
multipliers, and forms the new counter from the high and low halves of those
products xor-ed with words 1 and 3 and the key; the key advances by the two
Weyl increments between rounds.

Element layout (identical to the one documented in gmrf.h):
  block q, stream s, seed k: counter (q lo, q hi, s lo, s hi), key (k lo, k hi)
  normals   : pair q gives elements 2q, 2q+1 by Box-Muller from the 53-bit
              uniforms of words (w1:w0) and (w3:w2)
  Rademacher: element e is bit e % 128 of block e // 128 (+1 if set).
  Gamma     : element e, attempt t (t = 0..63) uses blocks 128 e + 2 t (a
              Box-Muller normal x from the cosine branch) and 128 e + 2 t + 1
              (the acceptance uniform u from words (w1:w0); for shape < 1 the
              boost uniform from words (w3:w2) of attempt 0); Marsaglia and
              Tsang's squeeze and log tests; after 64 rejections the value is
              d = shape - 1/3 (for shape >= 1).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(q: np.ndarray, seed: int, stream: int) -> np.ndarray:
    """Words (n, 4) uint32 of blocks q (array of block indices)."""
    q = np.asarray(q, dtype=np.uint64)
    c0 = q & MASK32
    c1 = q >> np.uint64(32)
    c2 = np.full_like(q, np.uint64(stream & 0xFFFFFFFF))
    c3 = np.full_like(q, np.uint64((stream >> 32) & 0xFFFFFFFF))
    k0 = seed & 0xFFFFFFFF
    k1 = (seed >> 32) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def uniform53(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    m = ((hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)) >> np.uint64(11)
    return (m.astype(np.float64) + 0.5) * 2.0 ** -53


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    pairs = (n + 1) // 2
    w = philox4x32_10(np.arange(pairs, dtype=np.uint64), seed, stream)
    u1 = uniform53(w[:, 0], w[:, 1])
    u2 = uniform53(w[:, 2], w[:, 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * pairs)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:n]


def rademacher(seed: int, stream: int, n: int) -> np.ndarray:
    blocks = (n + 127) // 128
    w = philox4x32_10(np.arange(blocks, dtype=np.uint64), seed, stream)
    e = np.arange(n)
    bits = (w[e // 128, (e % 128) // 32] >> (e % 32).astype(np.uint32)) & 1
    return np.where(bits == 1, 1, -1).astype(np.int8)


GAMMA_ATTEMPTS = 64


def gamma(seed: int, stream: int, shape: float, scale: np.ndarray) -> np.ndarray:
    """Gamma(shape, scale) variates, one per entry of scale, by the rejection
    method of Marsaglia and Tsang ("A simple method for generating gamma
    variables", ACM TOMS 26, 2000): with d = a - 1/3 and c = 1/sqrt(9 d), draw
    x ~ N(0, 1), v = (1 + c x)^3, keep d v when v > 0 and either
    u < 1 - 0.0331 x^4 or log u < x^2/2 + d (1 - v + log v); for a < 1, draw
    with a + 1 and multiply by U^(1/a)."""
    scale = np.asarray(scale, dtype=np.float64).ravel()
    n = scale.size
    a = float(shape) if shape >= 1.0 else float(shape) + 1.0
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    out = np.full(n, d)
    done = np.zeros(n, dtype=bool)
    e = np.arange(n, dtype=np.uint64)
    for t in range(GAMMA_ATTEMPTS):
        todo = np.flatnonzero(~done)
        if todo.size == 0:
            break
        qa = e[todo] * np.uint64(128) + np.uint64(2 * t)
        wa = philox4x32_10(qa, seed, stream)
        wb = philox4x32_10(qa + np.uint64(1), seed, stream)
        u1 = uniform53(wa[:, 0], wa[:, 1])
        u2 = uniform53(wa[:, 2], wa[:, 3])
        x = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        u = uniform53(wb[:, 0], wb[:, 1])
        v = (1.0 + c * x) ** 3
        ok = v > 0.0
        vs = np.where(ok, v, 1.0)
        acc = ok & ((u < 1.0 - 0.0331 * x ** 4) | (np.log(u) < 0.5 * x * x + d * (1.0 - vs + np.log(vs))))
        idx = todo[acc]
        out[idx] = d * vs[acc]
        done[idx] = True
    if shape < 1.0:
        wb = philox4x32_10(e * np.uint64(128) + np.uint64(1), seed, stream)
        out = out * uniform53(wb[:, 2], wb[:, 3]) ** (1.0 / shape)
    return out * scale
