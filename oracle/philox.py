"""Philox4x32-10 and the Metropolis random numbers drawn from it.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the host side of
the counter-based generator that the sampler uses when the caller passes no
explicit random numbers, written from the generator's published definition
(Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32 x 32 -> 64-bit
multiplications with the constants 0xD2511F53 and 0xCD9E8D57 on a 128-bit
counter, the 64-bit key bumped by the Weyl constants 0x9E3779B9 and
0xBB67AE85 between rounds.  Pinned by the published known-answer vectors in
tests/golden/philox4x32_10_kat.txt.

Draws of one Metropolis proposal (sweep t of a call with counter base c0,
electron e, walker w): three blocks b = 0, 1, 2 with counter (w, e + 2^16 b,
lo32(c0 + t), hi32(c0 + t)) and key (lo32(seed), hi32(seed)); each pair of
32-bit outputs (a, b) gives the uniform ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53
in (0, 1); u1..u4 from blocks 0 and 1 feed two Box-Muller pairs, of which
the first three normals are the step xi, and the first uniform of block 2 is
the acceptance draw.
"""
import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or ints) of 32-bit words, key: 2; returns 4 uint64
    arrays holding the 32-bit output words."""
    c = [np.asarray(x, dtype=np.uint64) for x in ctr]
    k = [np.asarray(x, dtype=np.uint64) for x in key]
    for r in range(10):
        if r:
            k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> _S32) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> _S32) ^ c[3] ^ k[1], p0 & _MASK]
    return c


def _unit(a, b):
    return ((a >> np.uint64(5)).astype(np.float64) * 67108864.0 + (b >> np.uint64(6)).astype(np.float64) + 0.5) \
        * (2.0 ** -53)


def sweep_randoms(seed: int, counter: int, t: int, n: int, W: int):
    """(xi [n][W][3], u [n][W]) of sweep t of a call with key seed and counter
    base counter."""
    e, w = np.meshgrid(np.arange(n, dtype=np.uint64), np.arange(W, dtype=np.uint64), indexing="ij")
    ct = (int(counter) + int(t)) & 0xFFFFFFFFFFFFFFFF
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    outs = []
    for b in range(3):
        ctr = (w, e + np.uint64(b << 16), np.uint64(ct & 0xFFFFFFFF), np.uint64(ct >> 32))
        outs.append(philox4x32_10(ctr, key))
    u1, u2 = _unit(outs[0][0], outs[0][1]), _unit(outs[0][2], outs[0][3])
    u3, u4 = _unit(outs[1][0], outs[1][1]), _unit(outs[1][2], outs[1][3])
    ua = _unit(outs[2][0], outs[2][1])
    r1, r2 = np.sqrt(-2.0 * np.log(u1)), np.sqrt(-2.0 * np.log(u3))
    xi = np.stack([r1 * np.cos(2.0 * np.pi * u2), r1 * np.sin(2.0 * np.pi * u2), r2 * np.cos(2.0 * np.pi * u4)], -1)
    return xi, ua
