"""Counter-based normal fields (oracle side), written from the published
definition of Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random
numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller transform.

Element i: counter (i mod 2^32, i div 2^32, 0, 0), key (seed mod 2^32,
seed div 2^32); ten rounds, each
    (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) after every round.  u_k = (x_k + 1/2) 2^-32;
E = sqrt(-2 ln u0) exp(2 pi i u1), E_adj = sqrt(-2 ln u2) exp(2 pi i u3).
Computed here in FP64 (the GPU draws in FP32; they agree to FP32 rounding).

Pinned by tests/test_oracle_philox.py against the known-answer vectors of the
Random123 distribution for Philox4x32-10.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def fields(shape, seed):
    """E, E_adj (complex128) of the given shape for `seed`."""
    n = int(np.prod(shape))
    i = np.arange(n, dtype=np.uint64)
    x = philox4x32_10(i & MASK, i >> np.uint64(32), 0, 0, seed & 0xFFFFFFFF, seed >> 32)
    u = [(xk.astype(np.float64) + 0.5) * 2.0 ** -32 for xk in x]
    r0, r1 = np.sqrt(-2.0 * np.log(u[0])), np.sqrt(-2.0 * np.log(u[2]))
    E = r0 * np.exp(2j * np.pi * u[1])
    A = r1 * np.exp(2j * np.pi * u[3])
    return E.reshape(shape), A.reshape(shape)
