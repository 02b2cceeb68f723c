"""Seeded synthetic matrix pairs (input construction only).

This module builds the inputs that the GPU path and the CPU oracle both
consume; it contains none of the randomized-GSVD arithmetic.  Library
primitives (a Gaussian generator, a QR to orthonormalise Gaussian factors, a
matrix product) are used only to construct the pairs.

Workload recipes (sizes follow the configurations the library is measured on):

* ``lowrank_pair``: G_i = U_i diag(s_i) Z^T + sigma_i N_i with a shared
  orthonormal Z (n x r), orthonormal U_i (m_i x r), decays s_i and iid
  Gaussian noise N_i.  The noise level is given either per entry or as a
  spectral floor nu, read as per-entry sigma = nu / (sqrt(m_i) + sqrt(n)) so
  that ||sigma N||_2 ~ nu.
* ``planted_gmp``: the real version of the paper's synthetic generator
  (Sec. 4.1): G1 = U* S1* R*, G2 = V* S2* R* with R* an n x n Gaussian,
  U*, V* orthonormalised Gaussians and planted alpha*, beta* with
  alpha*^2 + beta*^2 = 1, ranks 60% of min(m, p, n), middle alphas sorted
  uniform draws.  Requires m, p >= n (tall shapes).
"""
import math

import numpy as np


def _orth(rng, rows, cols):
    q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q


def lowrank_pair(m, p, n, r, s1, s2, seed, noise_entry=None, noise_spectral=None,
                 dtype=np.float64):
    """Return (G1, G2) as C-contiguous host arrays of ``dtype``."""
    rng = np.random.default_rng(seed)
    s1 = np.asarray(s1, dtype=np.float64)
    s2 = np.asarray(s2, dtype=np.float64)
    Z = _orth(rng, n, r)
    out = []
    for rows, s in ((m, s1), (p, s2)):
        U = _orth(rng, rows, r)
        G = (U * s[None, :]) @ Z.T
        if noise_spectral is not None:
            sig = noise_spectral / (math.sqrt(rows) + math.sqrt(n))
        else:
            sig = 0.0 if noise_entry is None else noise_entry
        if sig:
            G += sig * rng.standard_normal((rows, n))
        out.append(np.ascontiguousarray(G.astype(dtype)))
    return out[0], out[1]


def lowrank_pair_device(m, p, n, r, s1, s2, seed, noise_spectral, device, dtype=None):
    """The recipe of lowrank_pair (spectral noise floor) drawn on a torch
    device from torch's seeded generator, for pairs too large to build on
    the host quickly; returns (G1, G2) device tensors (float32 unless dtype
    is given).  Not the same numbers as lowrank_pair for the same seed."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(device=device, dtype=torch.float64)
    Z = torch.linalg.qr(torch.randn(n, r, generator=g, **f64))[0]
    out = []
    for rows, s in ((m, s1), (p, s2)):
        U = torch.linalg.qr(torch.randn(rows, r, generator=g, **f64))[0]
        G = (U * torch.as_tensor(np.asarray(s, dtype=np.float64), **f64)) @ Z.T
        G += (noise_spectral / (math.sqrt(rows) + math.sqrt(n))) * torch.randn(rows, n, generator=g, **f64)
        out.append(G.to(dtype).contiguous())
        del G, U
    return out[0], out[1]


def planted_gmp(m, p, n, seed, frac=0.6, dtype=np.float64, frac2=None):
    """Paper-style exactly low-rank GMP; returns (G1, G2, alpha*, beta*).
    Ranks frac min(m, p, n) for G1 and frac2 (default frac) of it for G2."""
    if m < n or p < n:
        raise ValueError("planted_gmp needs m >= n and p >= n")
    rng = np.random.default_rng(seed)
    nn = min(m, p, n)
    r1 = max(1, int(round(frac * nn)))
    r2 = max(1, int(round((frac if frac2 is None else frac2) * nn)))
    n_one = n - r2            # alpha = 1, beta = 0
    n_zero = n - r1           # alpha = 0, beta = 1
    s = n - n_one - n_zero
    if s < 0:
        raise ValueError("ranks too small for a GMP")
    mid = np.sort(rng.uniform(0.0, 1.0, size=s))[::-1]
    alpha = np.concatenate([np.ones(n_one), mid, np.zeros(n_zero)])
    beta = np.sqrt(np.maximum(0.0, 1.0 - alpha * alpha))
    Rs = rng.standard_normal((n, n))
    Us = _orth(rng, m, n)
    Vs = _orth(rng, p, n)
    G1 = (Us * alpha[None, :]) @ Rs
    G2 = (Vs * beta[None, :]) @ Rs
    return (np.ascontiguousarray(G1.astype(dtype)),
            np.ascontiguousarray(G2.astype(dtype)), alpha, beta)


# ------------------------------------------------------- named workloads ---
def small_fp64_pair(seed=101):
    """1000 x 300 and 800 x 300 FP64, rank 20, decays 0.8^j / 0.7^j, noise 1e-6
    per entry; sized k = 20, oversampling 10, one power iteration."""
    j = np.arange(20)
    G1, G2 = lowrank_pair(1000, 800, 300, 20, 0.8 ** j, 0.7 ** j, seed,
                          noise_entry=1e-6, dtype=np.float64)
    return dict(G1=G1, G2=G2, k=20, oversample=10, q=1, seed=1,
                name="pair 1000/800x300 fp64 rank20")


def medium_fp32_pair(seed=102, m=20000, p=15000, n=5000, r=100, decay2=None):
    """20000 x 5000 and 15000 x 5000 FP32, shared rank 100, decay 0.95 per
    index (both matrices unless decay2 is given), spectral noise floor 1e-4;
    k = 100, oversampling 10, two power iterations."""
    j = np.arange(r)
    s2 = (0.95 if decay2 is None else decay2) ** j
    G1, G2 = lowrank_pair(m, p, n, r, 0.95 ** j, s2, seed,
                          noise_spectral=1e-4, dtype=np.float32)
    return dict(G1=G1, G2=G2, k=r, oversample=10, q=2, seed=2,
                name=f"pair {m}/{p}x{n} fp32 rank{r}")


def large_fp32_pair(seed=103, m=100000, p=80000, n=2000, r=200, decay2=None):
    """100000 x 2000 and 80000 x 2000 FP32, rank 200, decay 0.97 per index,
    spectral noise floor 1e-3; k = 200, oversampling 20, two power iterations."""
    j = np.arange(r)
    s2 = (0.97 if decay2 is None else decay2) ** j
    G1, G2 = lowrank_pair(m, p, n, r, 0.97 ** j, s2, seed,
                          noise_spectral=1e-3, dtype=np.float32)
    return dict(G1=G1, G2=G2, k=r, oversample=20, q=2, seed=3,
                name=f"pair {m}/{p}x{n} fp32 rank{r}")


def batch_specs(npairs=256, seed=104, m_range=(2000, 20000), n_range=(50, 500),
                r_range=(10, 50), d_range=(0.6, 0.95), noise=1e-5):
    """Sizes and decays of a batch of uneven pairs (no matrices built).

    k_i = max(1, min(r_i, #{j : sqrt(s1_j^2 + s2_j^2) >= 10 noise (sqrt(max(m,p)) + sqrt(n))}))
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(npairs):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        p = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        r = int(rng.integers(r_range[0], min(r_range[1], n) + 1))
        d1 = float(rng.uniform(*d_range))
        d2 = float(rng.uniform(*d_range))
        j = np.arange(r)
        mag = np.sqrt(d1 ** (2 * j) + d2 ** (2 * j))
        thr = 10 * noise * (math.sqrt(max(m, p)) + math.sqrt(n))
        k = max(1, min(r, int(np.sum(mag >= thr))))
        specs.append(dict(m=m, p=p, n=n, r=r, d1=d1, d2=d2, noise=noise, k=k,
                          seed=seed * 100003 + i))
    return specs


def batch_pair(spec, dtype=np.float32):
    j = np.arange(spec["r"])
    return lowrank_pair(spec["m"], spec["p"], spec["n"], spec["r"],
                        spec["d1"] ** j, spec["d2"] ** j, spec["seed"],
                        noise_entry=spec["noise"], dtype=dtype)
