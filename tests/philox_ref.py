"""Host reference of the device normal generator (test infrastructure):
Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC11) keyed by the seed, counter = (pair index, 0, 0), and
the Box-Muller transform of the two 53-bit uniforms of its four output words.
Element e of the stream of a seed is the first (e even) or second (e odd)
normal of pair e // 2."""
import math

import numpy as np

_MASK = 0xFFFFFFFF
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr, key):
    c = [int(v) & _MASK for v in ctr]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0, p1 = _M0 * c[0], _M1 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 & _MASK, (p0 >> 32) ^ c[3] ^ k1, p0 & _MASK]
    return c


def normals(seed: int, offset: int, count: int) -> np.ndarray:
    out = np.empty(count)
    key = (seed & _MASK, seed >> 32)
    for i in range(count):
        e = offset + i
        pr = e >> 1
        c = philox4x32_10((pr & _MASK, pr >> 32, 0, 0), key)
        a = (c[0] << 32) | c[1]
        b = (c[2] << 32) | c[3]
        u = (a >> 11) * 2.0 ** -53 + 2.0 ** -54
        v = (b >> 11) * 2.0 ** -53
        rad = math.sqrt(-2.0 * math.log(u))
        out[i] = rad * (math.sin(2.0 * math.pi * v) if e & 1 else math.cos(2.0 * math.pi * v))
    return out
