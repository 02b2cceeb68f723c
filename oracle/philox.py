"""Counter-based Gaussian generator of the oracle (test infrastructure only).

The paper only asks for a standard Gaussian test matrix (Algorithm 1, the
block Omega_i of size n x b; Theorem "projector", Omega_1 of size n x (k+p)).
To let the GPU path and this oracle draw the *same* Omega from a seed, both
sides implement, separately, one published counter-based generator:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): a 10-round Feistel-like bijection on a 128-bit counter
  under a 64-bit key, multipliers 0xD2511F53 / 0xCD9E8D57 and key increments
  (Weyl constants) 0x9E3779B9 / 0xBB67AE85.
* Box-Muller (Box & Muller, 1958) turning two uniforms into two normals.

Layout of Omega (the reading this project takes, since the paper is silent):
  key      = (seed mod 2^32, seed >> 32)
  counter  = (row r, global column c >> 2, stream, 0)
  outputs (x0, x1) -> columns 4j, 4j+1 ; (x2, x3) -> columns 4j+2, 4j+3
  for a pair (xa, xb):  u1 = (xa + 1) 2^-32 in (0, 1],  u2 = xb 2^-32 in [0, 1)
                        z_even = sqrt(-2 ln u1) cos(2 pi u2)
                        z_odd  = sqrt(-2 ln u1) sin(2 pi u2)
Columns are indexed globally, so a fixed-size Omega with l columns is the
prefix of the stream the adaptive loop walks block by block (the proof of
Lemma c2 views the blocks Omega_i as consecutive column blocks of one n x n
Gaussian matrix), and a 16-column probe is again a prefix.

Stream ids: 1 = Omega for G1, 2 = Omega for G2.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.
"""
import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_G1 = 1
STREAM_G2 = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on uint32 arrays (broadcastable).

    One round maps (c0, c1, c2, c3) under key (k0, k1) to
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
    the key is bumped by the Weyl constants between rounds.
    Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = PHILOX_M0 * c0          # < 2^64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def raw_bits(seed, stream, n_rows, col0, ncols):
    """The uint32 words feeding columns [col0, col0+ncols) of rows 0..n_rows-1.

    Returns an (n_rows, ncols) uint32 array where entry (r, c) is the word that
    lands on column c: x0/x1/x2/x3 of counter (r, c >> 2, stream, 0) for
    c mod 4 = 0/1/2/3.  (The Box-Muller pairing is (x0,x1) and (x2,x3).)
    """
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    cols = np.arange(col0, col0 + ncols, dtype=np.int64)
    j = np.unique(cols >> 2)
    r = np.arange(n_rows, dtype=np.uint64)[:, None]
    x = philox4x32_10(r, j[None, :].astype(np.uint64), np.uint64(stream),
                      np.uint64(0), k0, k1)
    words = np.stack(x, axis=-1)                   # (n_rows, len(j), 4)
    jpos = (cols >> 2) - j[0]
    return words[:, jpos, cols & 3]


def gaussian_matrix(seed, stream, n_rows, col0, ncols):
    """Omega[r, c] for r < n_rows, col0 <= c < col0+ncols, in float64.

    Each Box-Muller pair is evaluated in float64 from the exact uniforms.
    """
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    if ncols <= 0 or n_rows <= 0:
        return np.zeros((max(n_rows, 0), max(ncols, 0)))
    j0 = col0 >> 2
    j1 = (col0 + ncols - 1) >> 2
    j = np.arange(j0, j1 + 1, dtype=np.uint64)
    r = np.arange(n_rows, dtype=np.uint64)[:, None]
    x0, x1, x2, x3 = philox4x32_10(r, j[None, :], np.uint64(stream),
                                   np.uint64(0), k0, k1)
    two32 = 2.0 ** -32
    out = np.empty((n_rows, len(j), 4))
    for (xa, xb, ce, co) in ((x0, x1, 0, 1), (x2, x3, 2, 3)):
        u1 = (xa.astype(np.float64) + 1.0) * two32
        u2 = xb.astype(np.float64) * two32
        rad = np.sqrt(-2.0 * np.log(u1))
        ang = 2.0 * np.pi * u2
        out[:, :, ce] = rad * np.cos(ang)
        out[:, :, co] = rad * np.sin(ang)
    full = out.reshape(n_rows, 4 * len(j))
    start = col0 - 4 * int(j0)
    return np.ascontiguousarray(full[:, start:start + ncols])
