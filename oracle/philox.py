"""Philox4x32-10, the oracle's own copy (test infrastructure only).

Written from the generator's published definition (Salmon et al., SC'11,
section on Philox): a 4x32-bit counter and a 2x32-bit key; each round
multiplies counter words 0 and 2 by two fixed odd constants, splits each 64-bit
product into high and low halves, and forms the new counter as

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),

after which the key is bumped by two Weyl constants.  Ten rounds are applied.
Pinned by the published known-answer vectors (tests/golden/philox4x32_10_kat.txt).

The MCSF draws X ~ B(N, 1/2) per (term, channel) (Proposition 2, Algorithm 1
"Draw X").  The paper leaves the generator unspecified; this project draws the
N Bernoulli(1/2) bits of X from Philox words keyed by the seed, with counter
(t, m, block, 0) -- see ``oracle.mcsf.draw_binomial``.
"""

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Apply Philox4x32 with 10 rounds.

    ctr : array (n, 4) of uint32 counters (or a single length-4 sequence)
    key : length-2 sequence of uint32
    returns array (n, 4) of uint32 outputs
    """
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _SH32, p0 & _MASK32
        hi1, lo1 = p1 >> _SH32, p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)
