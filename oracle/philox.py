"""Counter-based Gaussian draws for the simulations (test infrastructure only).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit counter and a
2x32-bit key, ten rounds, each round two 32x32->64-bit products with the
multipliers 0xD2511F53 and 0xCD9E8D57, and a Weyl key schedule with increments
0x9E3779B9 and 0xBB67AE85.  Pinned by the known-answer vectors the authors
publish with their reference distribution (tests/golden/philox4x32_10_kat.txt).

Normals come from the Box-Muller transform (Box & Muller 1958) of pairs of
uniforms u = (x + 1/2) 2^-32, evaluated in float64.

Stream layout for simulation `i` with 64-bit `seed`: key = (seed mod 2^32,
seed div 2^32); normal number q uses counter (q div 4, i, 0, 0); outputs
(x0, x1) give normals 4(q div 4) + {0, 1} (cos, sin), (x2, x3) give + {2, 3}.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr [..., 4] uint32, key [2] uint32 -> [..., 4] uint32."""
    c = [ctr[..., i].astype(np.uint64) for i in range(4)]
    k0 = np.uint64(np.uint32(key[0]))
    k1 = np.uint64(np.uint32(key[1]))
    for rnd in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [(hi1 ^ c[1] ^ k0) & _MASK, lo1, (hi0 ^ c[3] ^ k1) & _MASK, lo0]
        k0 = (k0 + np.uint64(_W0)) & _MASK
        k1 = (k1 + np.uint64(_W1)) & _MASK
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def uniforms(x: np.ndarray) -> np.ndarray:
    return (x.astype(np.float64) + 0.5) * (2.0 ** -32)


def normals_for_sim(seed: int, sim: int, count: int) -> np.ndarray:
    """`count` (a multiple of 4) standard normals of simulation `sim`, float64."""
    assert count % 4 == 0
    nblk = count // 4
    ctr = np.zeros((nblk, 4), np.uint32)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] = np.uint32(sim)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32)
    x = philox4x32_10(ctr, key)
    u = uniforms(x)
    out = np.empty((nblk, 4))
    for a in (0, 2):
        r = np.sqrt(-2.0 * np.log(u[:, a]))
        ang = 6.283185307179586 * u[:, a + 1]
        out[:, a] = r * np.cos(ang)
        out[:, a + 1] = r * np.sin(ang)
    return out.reshape(-1)


def draws_for_sims(seed: int, sims, n: int, ncomp: int) -> np.ndarray:
    """[len(sims)][2][ncomp][n][n] normals in the layout the simulations consume."""
    per = 2 * ncomp * n * n
    return np.stack([normals_for_sim(seed, int(i), per).reshape(2, ncomp, n, n) for i in sims])
