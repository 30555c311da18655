"""Philox4x32-10 counter-based generator and the uniform-double mapping.

Oracle code (test infrastructure only).

Generator: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit key; ten rounds of two
32x32->64 multiplications with the round-key bumped by the Weyl constants.
The paper under study uses this generator for its "Calc 2".

Stream layout: key = (seed, tag); counter = (block, graph, sample_lo,
sample_hi).  One block yields two uniform doubles: (x0, x1) and (x2, x3).
A uniform double in (0, 1) from two words (a, b) is
(2 k + 1) * 2^-53 with k = (a >> 6) * 2^26 + (b >> 6) < 2^52: exact in
binary64, never 0 or 1.
"""
MASK = 0xFFFFFFFF
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def u01(a, b):
    k = (a >> 6) * 67108864 + (b >> 6)
    return (2 * k + 1) * (1.0 / 9007199254740992.0)


def uniforms(seed, tag, graph, sample, count):
    """The first ``count`` uniforms of one sample's stream."""
    out = []
    blk = 0
    key = (seed & MASK, tag & MASK)
    while len(out) < count:
        x = philox4x32_10((blk, graph & MASK, sample & MASK, (sample >> 32) & MASK), key)
        out.append(u01(x[0], x[1]))
        out.append(u01(x[2], x[3]))
        blk += 1
    return out[:count]
