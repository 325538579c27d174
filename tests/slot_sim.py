"""Slot-level simulator of Alg. 1 and Alg. 2 in plain float64.

A ciphertext is replaced by the real vector it encrypts, Add by `+`, Mul by
`*`, Rot(v, r) by `np.roll(v, -r)` (slot j receives slot j + r) and Res by
the identity.  It pins the index logic of the oracle's Blind-Match layer
independently of any encryption.
"""
import numpy as np


def rot(v, r):
    return np.roll(v, -r)


def expand(qslots, d, k):
    c = d // k
    n = qslots.size
    s = np.arange(n)
    out = []
    for i in range(k):
        ci = qslots * (((s % d) // c) == i)
        for t in range(int(np.log2(k))):
            r = c << t
            step = -r if ((i >> t) & 1) == 0 else r
            ci = ci + rot(ci, step)
        out.append(ci)
    return out


def hec3(cu, cs, d, k):
    c = d // k
    acc = np.zeros_like(cu[0])
    for i in range(k):
        acc = acc + cu[i] * cs[i]
    for t in range(int(np.log2(c))):
        acc = acc + rot(acc, 1 << t)
    return acc
