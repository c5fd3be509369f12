"""Philox4x32-10 and the Gaussian sketch of the bond swap (test infrastructure only).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
32x32->64 multiplications with the constants M0 = 0xD2511F53 and
M1 = 0xCD9E8D57, the Weyl key schedule W0 = 0x9E3779B9, W1 = 0xBB67AE85.

Sketch entries (the random tensor Omega of App. A) are standard normals made
by Box-Muller from the first two output words of one Philox call:
    u1 = (x0 + 1/2) 2^-32,  u2 = (x1 + 1/2) 2^-32,
    z  = sqrt(-2 ln u1) cos(2 pi u2).
Entry Omega[beta, j_t1, j_t2, j_t3, m] drawn at RG step k uses the counter
    c0 = j_t1 | j_t2 << 8 | j_t3 << 16 | beta << 24
    c1 = m | k << 16
    c2 = instance,  c3 = 0x4F4D4547 ("OMEG")
and the key (seed mod 2^32, seed >> 32).  The counter is a function of the
multi-index, not of a memory layout, so padding a leg does not change a draw.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
TAG = 0x4F4D4547
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. Counter words are uint32 arrays; returns 4 uint32 arrays."""
    x0 = np.asarray(c0, dtype=np.uint64)
    x1 = np.asarray(c1, dtype=np.uint64)
    x2 = np.asarray(c2, dtype=np.uint64)
    x3 = np.asarray(c3, dtype=np.uint64)
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    key0 = np.uint64(k0 & MASK)
    key1 = np.uint64(k1 & MASK)
    m = np.uint64(MASK)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd > 0:
            key0 = np.uint64((int(key0) + W0) & MASK)
            key1 = np.uint64((int(key1) + W1) & MASK)
        p0 = np.uint64(M0) * x0
        p1 = np.uint64(M1) * x2
        hi0, lo0 = p0 >> s32, p0 & m
        hi1, lo1 = p1 >> s32, p1 & m
        x0, x1, x2, x3 = (hi1 ^ x1 ^ key0), lo1, (hi0 ^ x3 ^ key1), lo0
    return tuple(x.astype(np.uint32) for x in (x0, x1, x2, x3))


def box_muller(x0, x1):
    """Standard normal from two uint32 words (cosine branch of Box-Muller)."""
    u1 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def sketch_omega(seed, step, instance, chi, jdims, m):
    """Gaussian Omega[beta, j_t1, (j_t2, (j_t3,)) m] for the bond swap of RG step ``step``.

    ``jdims`` holds the dims of the transverse backward legs (1 to 3 of them).
    """
    jd = list(jdims) + [1] * (3 - len(jdims))
    b = np.arange(chi, dtype=np.uint64).reshape(chi, 1, 1, 1, 1)
    j1 = np.arange(jd[0], dtype=np.uint64).reshape(1, jd[0], 1, 1, 1)
    j2 = np.arange(jd[1], dtype=np.uint64).reshape(1, 1, jd[1], 1, 1)
    j3 = np.arange(jd[2], dtype=np.uint64).reshape(1, 1, 1, jd[2], 1)
    mm = np.arange(m, dtype=np.uint64).reshape(1, 1, 1, 1, m)
    c0 = j1 | (j2 << np.uint64(8)) | (j3 << np.uint64(16)) | (b << np.uint64(24))
    c1 = mm | np.uint64((step & 0xFFFF) << 16)
    c2 = np.uint64(instance & MASK)
    c3 = np.uint64(TAG)
    x0, x1, _x2, _x3 = philox4x32_10(c0, c1, c2, c3, seed & MASK, (seed >> 32) & MASK)
    z = box_muller(x0, x1)
    return z.reshape([chi] + list(jdims) + [m])
