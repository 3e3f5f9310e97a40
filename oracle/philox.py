"""Philox-4x32-10 counter-based generator (test infrastructure).

Written from the published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a
2-word key go through 10 rounds of

    (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))

with multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the
Weyl constants W0 = 0x9E3779B9, W1 = 0xBB67AE85 between rounds.  Pure Python
integers, so the output is exact.  The sampler's device draws are checked
against this bit for bit.
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32(ctr, key, rounds: int = 10):
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK, (p0 >> 32) ^ c3 ^ k1, p0 & MASK)
    return (c0, c1, c2, c3)
