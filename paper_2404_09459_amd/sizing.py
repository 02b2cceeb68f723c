"""Learned sketch sizing: probe features, labels from the method itself, and
training of the 32-64-64-2 network with the library's own HIP kernels.

The network reads the 32 features of a pair (per matrix: eight normalised
singular values of the 16-column probe G_i Omega[:, :16] and eight entries of
the R-diagonal profile of the widest sketch at columns placed relative to k,
as log10 ratios) and regresses
(log2(l / k), q): the sketch width relative to the target rank and the power
count.  A pair's label is the cheapest point of the grid
l in {k+4, k+8, k+16, k+32, 2k} x q in {0..3} (fewest passes over G, then the
smallest l) at which the production (mixed-precision) run meets the angular
tolerance against a converged FP64 run of the same method
(l_ref = min(2k + 50, cap), q_ref = 4) on the pairs whose weaker component
is above the noise floor.  The network is not in the paper.
"""
import ctypes
import math

import numpy as np

from . import inputs as I
from . import rgsvd as R

GRID_Q = (0, 1, 2, 3)
TOL_THETA = 1e-4
LABEL_MARGIN = 0.1
# training pairs: the learned-sizing workload's ranks (up to 220 shared
# components, n up to 1000) on fewer rows (m, p <= 4000), so that labelling
# stays a few seconds of GPU time while the probe spectra cover the
# workload's (a 16-column probe of a rank-200 pair is nearly flat).  The
# decays follow from the magnitude of the last shared component, so that
# about half of the pairs keep all r components above the noise floor
# (those are the pairs with a gap at k, the ones the labels can judge), and
# k counts the components above twice the floor, so that tails a few times
# the noise (where more passes pay) are among them.  The two decays are
# drawn apart: with one decay for both matrices every GSV sits near
# 1/sqrt(2) and theta is set by how the noise splits between G1 and G2,
# which no sketch size makes more exact
TRAIN_RANGES = dict(m_range=(1000, 4000), n_range=(200, 1000), r_range=(5, 220), tail_range=(1e-4, 0.3),
                    k_floor=2.0)
# a few training pairs at the workload's own scale (drawn on the device):
# the noise a sketch takes in grows with the rows and n, and with it the
# passes a tail near the floor needs
TRAIN_LARGE = dict(m_range=(20000, 100000), n_range=(1000, 2000), r_range=(50, 220), tail_range=(1e-4, 0.3),
                   k_floor=2.0)


def _torch():
    import torch
    return torch


# ------------------------------------------------------------ features ---
def probe_features(G1, G2, seed, k, precision="fp64"):
    """The 32 sizing features of a device pair for target rank k (float32
    device tensor), from a learned plan of the pair's shapes, as a learned
    run of that precision computes them."""
    torch = _torch()
    m, n = G1.shape
    p = G2.shape[0]
    dt = R.F64 if G1.dtype == torch.float64 else R.F32
    plan = R.Plan(R.make_desc(m, p, n, k, 0, 0, seed, dt, precision, "learned"), G1.device)
    feat = torch.empty(32, dtype=torch.float32, device=G1.device)
    R.check(R.lib().rgsvd_probe_features(plan.h, R._ptr(G1), G1.stride(0), R._ptr(G2), G2.stride(0),
                                         plan.ws_ptr, R._ptr(feat), R._stream(G1.device)), "probe_features")
    torch.cuda.current_stream(G1.device).synchronize()
    del plan
    return feat


# ----------------------------------------------------------------- MLP ---
def init_params(seed, device):
    """He-initialised packed parameters (W[out][in] row-major per layer)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    dims = (32, 64, 64, 2)
    parts = []
    for i in range(3):
        fi, fo = dims[i], dims[i + 1]
        parts.append(rng.standard_normal(fo * fi) * math.sqrt(2.0 / fi) * (0.5 if i == 2 else 1.0))
        parts.append(np.zeros(fo))
    return torch.tensor(np.concatenate(parts), dtype=torch.float32, device=device)


def mlp_forward(params, X):
    torch = _torch()
    X = X.contiguous()
    B = X.shape[0]
    Y = torch.empty((B, 2), dtype=torch.float32, device=X.device)
    act = torch.empty((B, 128), dtype=torch.float32, device=X.device)
    R.check(R.lib().rgsvd_mlp_forward(R._ptr(params), R._ptr(X), B, R._ptr(Y), R._ptr(act),
                                      R._stream(X.device)), "mlp_forward")
    return Y, act


def mlp_backward(params, X, T, act):
    torch = _torch()
    B = X.shape[0]
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    R.check(R.lib().rgsvd_mlp_backward(R._ptr(params), R._ptr(X.contiguous()), R._ptr(T.contiguous()), B,
                                       R._ptr(act), R._ptr(g), R._ptr(loss), R._stream(X.device)),
            "mlp_backward")
    return g, loss


def adam(params, g, mom, vel, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    R.check(R.lib().rgsvd_mlp_adam(R._ptr(params), R._ptr(g), R._ptr(mom), R._ptr(vel), step,
                                   ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2),
                                   ctypes.c_float(eps), R._stream(params.device)), "mlp_adam")


def train(X, T, device, epochs=400, lr=3e-3, seed=0):
    """Full-batch Adam on (X, T) (device float32); returns params, losses."""
    torch = _torch()
    params = init_params(seed, device)
    mom = torch.zeros_like(params)
    vel = torch.zeros_like(params)
    losses = []
    for step in range(1, epochs + 1):
        _, act = mlp_forward(params, X)
        g, loss = mlp_backward(params, X, T, act)
        adam(params, g, mom, vel, step, lr=lr)
        if step % 50 == 0 or step == 1:
            losses.append(float(loss.item()))
    return params, losses


# --------------------------------------------------------------- pairs ---
def pair_specs(npairs, seed, m_range=(500, 3000), n_range=(100, 400), r_range=(5, 40),
               d_range=(0.5, 0.99), nu_range=(1e-6, 1e-2), tail_range=None, k_floor=10.0, p_same=0.0):
    """Training / held-out pairs shaped like the learned-sizing workload
    (scaled down): shared rank r, decays d1, d2, spectral noise floor nu
    (log-uniform); k = the number of shared components above k_floor nu
    (at least 2).
    With tail_range the decays are d_i = tau_i^(1/(r-1)) for tail magnitudes
    tau_i drawn log-uniform from it, else uniform from d_range; with
    probability p_same both matrices take d1."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(npairs):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        p = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        r = int(rng.integers(r_range[0], max(r_range[0], min(r_range[1], n // 4)) + 1))
        if tail_range is None:
            d1 = float(rng.uniform(*d_range))
            d2 = float(rng.uniform(*d_range))
        else:
            lo, hi = np.log(tail_range[0]), np.log(tail_range[1])
            d1, d2 = (float(np.exp(rng.uniform(lo, hi)) ** (1.0 / max(1, r - 1))) for _ in range(2))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        if p_same > 0.0 and rng.uniform() < p_same:
            d2 = d1
        j = np.arange(r)
        mag = np.minimum(d1 ** j, d2 ** j)
        k = int(max(2, min(r, np.sum(mag >= k_floor * nu))))
        out.append(dict(m=m, p=p, n=n, r=r, d1=d1, d2=d2, nu=nu, k=k, seed=seed * 7919 + i))
    return out


def make_pair_device(spec, device):
    """A pair of the spec drawn on the device (large held-out pairs)."""
    j = np.arange(spec["r"])
    return I.lowrank_pair_device(spec["m"], spec["p"], spec["n"], spec["r"], spec["d1"] ** j, spec["d2"] ** j,
                                 spec["seed"], spec["nu"], device)


def make_pair(spec):
    j = np.arange(spec["r"])
    return I.lowrank_pair(spec["m"], spec["p"], spec["n"], spec["r"], spec["d1"] ** j, spec["d2"] ** j,
                          spec["seed"], noise_spectral=spec["nu"], dtype=np.float32)


def _pinned(ref, k, nu):
    s = ref["sigma_B"]
    weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
    if len(s) > k and s[k - 1] < 2 * s[k]:
        return np.arange(0)
    return np.where(weak >= 10 * nu)[0]


def _run(g1, g2, k, l, q, seed, precision, timed=False, sizing="fixed", tol=0.0, block=0, lmax=0,
         model=None):
    """One run with a plan of its own (freed afterwards).  timed=True also
    returns the mean wall time (ms) of two more runs, HIP events around each
    on the device's stream, after the first."""
    torch = _torch()
    m, n = g1.shape
    p = g2.shape[0]
    dt = R.F64 if g1.dtype == torch.float64 else R.F32
    plan = R.Plan(R.make_desc(m, p, n, k, l - k, q, seed, dt, precision, sizing, "truncated", tol, block, lmax),
                  g1.device)
    if model is not None:
        R.check(R.lib().rgsvd_set_sizing_model(plan.h, R._ptr(model), R._stream(g1.device)), "set model")
    o = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, g1.device, uvr=(precision == "fp64"))
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    ms = None
    if timed:
        st = torch.cuda.current_stream(g1.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(2):
            R.run(plan, g1, g2, o)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 2
    out = {kk: v.cpu().numpy() for kk, v in o.items() if kk not in ("Ut", "Vt")}
    del plan
    return (out, ms) if timed else out


def l_grid(k, cap):
    return sorted({v for v in (min(cap, x) for x in (k + 4, k + 8, k + 16, k + 32, 2 * k)) if v >= k})


def passes(got, ref, idx, tol=TOL_THETA):
    """Whether the pinned angular distances are within tol; None when no
    index is pinned (nothing to judge: such pairs are counted apart)."""
    if len(idx) == 0:
        return None
    return float(np.max(np.abs(got["theta"][idx] - ref["theta"][idx]))) <= tol


def label(g1, g2, spec, seed=1, precision="mixed", margin=LABEL_MARGIN):
    """(l, q, reference, pinned indices) of a device pair: the cheapest grid
    point whose angular error is within margin * TOL_THETA.  The network
    regresses onto these points; a label on the pass boundary itself would
    put about half of the mispredicted pairs on the failing side, so the
    margin keeps the regression's scatter inside the tolerance.  A pair with
    no pinned index has no label (l = q = None)."""
    k, nu = spec["k"], spec["nu"]
    cap = min(spec["m"], spec["p"], spec["n"], 224)
    lref = min(2 * k + 50, cap)
    ref = _run(g1, g2, k, lref, 4, seed, "fp64")
    idx = _pinned(ref, k, nu)
    if len(idx) == 0:
        return None, None, ref, idx
    grid = l_grid(k, cap)
    for q in GRID_Q:
        for l in grid:
            if passes(_run(g1, g2, k, l, q, seed, precision), ref, idx, margin * TOL_THETA):
                return l, q, ref, idx
    return grid[-1], GRID_Q[-1], ref, idx


def label_set(dev, specs, make, seed=1, precision="mixed"):
    """Features and targets of the pinned pairs among specs (make(spec) gives
    the device pair); returns (X, T, number of unpinned pairs left out)."""
    X, T, skipped = [], [], 0
    for s in specs:
        g1, g2 = make(s)
        l, q, _, _ = label(g1, g2, s, seed=seed, precision=precision)
        if l is None:
            skipped += 1
        else:
            X.append(probe_features(g1, g2, seed, s["k"], precision=precision).cpu().numpy())
            T.append(targets(s["k"], l, q))
        del g1, g2
    return X, T, skipped


def cost(spec, l, q):
    """Passes over G (2q + 2), the HBM-bound cost of a run."""
    return 2 * q + 2


def targets(k, l, q):
    return (math.log2(l / k), float(q))


def decide(y, k, cap):
    """Same rounding as the library: the smallest grid l at or above
    k 2^y0; q = floor(y1 + 0.9) clamped to [0, 3]."""
    grid = l_grid(k, cap)
    want = k * 2.0 ** min(float(y[0]), 8.0)
    l = next((v for v in grid if v >= want), grid[-1])
    q = int(min(3, max(0, math.floor(float(y[1]) + 0.9))))
    return l, q
