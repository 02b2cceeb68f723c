"""FP64 CPU oracle of the learned-sizing features and labels (test
infrastructure only: tests, the smoke check and the benchmark's CPU-baseline
leg may import it).

Features of a pair: for each matrix, the 16 singular values of the probe
sketch G Omega[:, :16] (the first 16 columns of the matrix's own Omega stream,
so the probe is a prefix of every larger sketch), as log10(sigma_j / sigma_1)
floored at -8 (what an FP64 Gram of the probe resolves); G1's 16 values, then
G2's.  The sizing network is not in the
paper; these definitions are the build's reading of it.

Label grid: sketch size l in {k+4, k+8, k+16, k+32, 2k} (at most min(m, p, n)),
power count q in {0, 1, 2, 3}.  Targets of the network: (log2(l / k), q).
"""
import numpy as np

from .philox import gaussian_matrix

PROBE = 16
FLOOR = -8.0


def probe_spectrum(G, seed, stream):
    """Singular values of G Omega[:, :16] (descending)."""
    Om = gaussian_matrix(seed, stream, G.shape[1], 0, PROBE)
    return np.linalg.svd(np.asarray(G, dtype=np.float64) @ Om, compute_uv=False)


def features(G1, G2, seed):
    out = []
    for G, stream in ((G1, 1), (G2, 2)):
        s = probe_spectrum(G, seed, stream)
        f = np.full(PROBE, FLOOR)
        if s[0] > 0:
            with np.errstate(divide="ignore"):
                f = np.maximum(np.log10(s / s[0]), FLOOR)
        out.append(f)
    return np.concatenate(out)


def l_grid(k, cap):
    g = sorted({min(cap, v) for v in (k + 4, k + 8, k + 16, k + 32, 2 * k)})
    return [v for v in g if v >= k]


def decide(y, k, cap):
    """Network output (log2(l / k), q) -> (l, q): the smallest grid size at
    or above k 2^y0, and q rounded with a bias of 0.4 towards more passes
    (q >= 1 once y1 reaches 0.1)."""
    grid = l_grid(k, cap)
    want = k * 2.0 ** min(float(y[0]), 8.0)
    l = next((v for v in grid if v >= want), grid[-1])
    q = int(min(3, max(0, np.floor(float(y[1]) + 0.5 + 0.4))))
    return l, q
