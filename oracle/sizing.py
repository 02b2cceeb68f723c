"""FP64 CPU oracle of the learned-sizing features and labels (test
infrastructure only: tests, the smoke check and the benchmark's CPU-baseline
leg may import it).

Features of a pair (16 per matrix, G1's then G2's), all log10 ratios floored
at -8 (what an FP64 Gram of a sketch resolves):

* the probe: singular values s_2, s_4, ..., s_16 of the probe sketch
  G Omega[:, :16] (the first 16 columns of the matrix's own Omega stream, so
  the probe is a prefix of every larger sketch), as log10(s_j / s_1);
* the profile: the diagonal of the triangular factor R of the sketch
  G Omega[:, :L] at the widest grid width L = max(l_grid(k, cap)),
  rho_j = |R_jj| (the distance of sketch column j from the span of the
  columns before it), as log10(rho_j / rho_1) at the positions
  ceil(k/4), ceil(k/2), ceil(3k/4), k, k+4, k+8, k+16 and L (each clamped to
  [1, L]).  The probe sees the top of the spectrum, the profile where the
  rank-k part ends against the noise.

The sizing network is not in the paper; these definitions are the build's
reading of it.

Label grid: sketch size l in {k+4, k+8, k+16, k+32, 2k} (at most min(m, p, n)),
power count q in {0, 1, 2, 3}.  Targets of the network: (log2(l / k), q).
"""
import numpy as np

from .philox import gaussian_matrix

PROBE = 16
FLOOR = -8.0
PROBE_AT = (2, 4, 6, 8, 10, 12, 14, 16)     # 1-based indices of the probe's singular values kept


def probe_spectrum(G, seed, stream):
    """Singular values of G Omega[:, :16] (descending)."""
    Om = gaussian_matrix(seed, stream, G.shape[1], 0, PROBE)
    return np.linalg.svd(np.asarray(G, dtype=np.float64) @ Om, compute_uv=False)


def profile_positions(k, L):
    """1-based sketch columns the profile features read."""
    raw = (-(-k // 4), -(-k // 2), -(-3 * k // 4), k, k + 4, k + 8, k + 16, L)
    return [min(max(1, v), L) for v in raw]


def sketch_profile(G, seed, stream, L):
    """|R_jj| of the triangular factor of G Omega[:, :L] (j = 1..L)."""
    Om = gaussian_matrix(seed, stream, G.shape[1], 0, L)
    R = np.linalg.qr(np.asarray(G, dtype=np.float64) @ Om, mode="r")
    return np.abs(np.diag(R))


def _log_ratio(v, v0):
    if not v0 > 0:
        return np.full(len(v), FLOOR)
    with np.errstate(divide="ignore"):
        return np.maximum(np.log10(np.asarray(v) / v0), FLOOR)


def features(G1, G2, seed, k, cap):
    """The 32 features of a pair for target rank k and width cap."""
    L = max(l_grid(k, cap))
    pos = np.array(profile_positions(k, L)) - 1
    out = []
    for G, stream in ((G1, 1), (G2, 2)):
        s = probe_spectrum(G, seed, stream)
        rho = sketch_profile(G, seed, stream, L)
        out.append(_log_ratio(s[np.array(PROBE_AT) - 1], s[0]))
        out.append(_log_ratio(rho[pos], rho[0]))
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
