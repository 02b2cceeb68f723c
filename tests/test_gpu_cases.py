"""Special cases of the method on the GPU against the CPU oracle and the
closed forms that pin them (FP64 arithmetic, through the C ABI).

* Full mode (t = n) on an exactly low-rank GMP built by the real form of the
  paper's synthetic generator (Sec. 4): Algorithm 2 as written, zero-appended
  alphas when l1 < n, against the oracle, the deterministic GSVD (Algorithm 2
  with Q1 = I, Q2 = I) and the planted alpha*; with fixed sizes, and with
  both bases built by Algorithm 1 (b = 100 and b = 16, unequal ranks).
* Disjoint row supports: every generalized singular pair is (1, 0) or
  (0, 1); the beta = 0 columns of V are zero and flagged.
* G1 = c G2: one cluster alpha = c / sqrt(1 + c^2), theta = arctan(c) - pi/4,
  D = 1 (the closed forms of Sec. 1's quantities for equal spectra).
* Numerically rank-deficient sketches (rank(G) < l): CholeskyQR needs its
  shift and says so; the dominant pairs still match the oracle.
* A NaN in G: the run ends, flags FLAG_NONFINITE and returns NaN GSVs.
Where columns of U, V, R are not unique (ties, clusters), the reconstruction
G_i = U diag(alpha) R, G_i = V diag(beta) R is checked instead.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_09459_amd import rgsvd as R
    R.lib()
    return torch.device("cuda:0")


def _run(dev, G1, G2, k, o, q, seed, mode="truncated", precision="fp64"):
    from paper_2404_09459_amd import rgsvd as R
    g1 = torch.from_numpy(np.ascontiguousarray(G1)).to(dev)
    g2 = torch.from_numpy(np.ascontiguousarray(G2)).to(dev)
    r = R.rgsvd(g1, g2, k, o, q, seed, precision=precision, mode=mode)
    torch.cuda.synchronize()
    return {kk: v.cpu().numpy() for kk, v in r.items()}


def _gsv_err(got, ref):
    return dict(alpha=float(np.max(np.abs(got["alpha"] - ref["alpha"]))),
                beta=float(np.max(np.abs(got["beta"] - ref["beta"]))),
                theta=float(np.max(np.abs(got["theta"] - ref["theta"]))),
                P=float(max(np.max(np.abs(got["P1"] - ref["P1"])), np.max(np.abs(got["P2"] - ref["P2"])))),
                D=float(np.max(np.abs(got["D"] - [ref["D1"], ref["D2"]]))))


def _recon(got, G1, G2):
    """Relative residuals of G1 = U diag(alpha) R and G2 = V diag(beta) R."""
    U, V, Rm = got["U"], got["V"], got["R"]
    r1 = np.linalg.norm(G1 - (U * got["alpha"]) @ Rm) / np.linalg.norm(G1)
    r2 = np.linalg.norm(G2 - (V * got["beta"]) @ Rm) / np.linalg.norm(G2)
    return r1, r2


def _flags(got):
    from paper_2404_09459_amd import rgsvd as R
    return R.decode_flags(int(got["info"][4]))


def _beta_zero_consistent(got):
    """beta < 1e-14 exactly where the V column is zero, and the flag with it."""
    bz = got["beta"] < 1e-14
    vz = np.all(got["V"] == 0.0, axis=0)
    assert np.array_equal(bz[~vz], np.zeros(np.sum(~vz), bool)), "nonzero V column with beta below 1e-14"
    assert np.all(vz[bz]), "V column of a beta below 1e-14 is not zero"
    assert ("beta_zero" in _flags(got)) == bool(np.any(bz))


@pytest.mark.parametrize("m,p,n,frac,k,o", [
    (300, 250, 150, 0.6, 80, 10),     # l1 = l2 = 90 = rank, l1 + l2 = 180 >= n
    (240, 200, 120, 0.75, 70, 20),    # l = 90 = rank, 60 alphas of the middle
])
def test_full_mode_planted_gmp(dev, m, p, n, frac, k, o):
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    G1, G2, a_star, b_star = I.planted_gmp(m, p, n, seed=31 + n, frac=frac)
    l = k + o
    _say(f"full mode: planted GMP {m}/{p}x{n}, ranks {int(round(frac * n))}, l={l}, t=n={n}")
    got = _run(dev, G1, G2, k, o, 1, 17, mode="full")
    ref = O.rgsvd(G1, G2, k, o, 1, 17, t=n)
    det = O.full_gsvd(G1, G2)
    e = _gsv_err(got, ref)
    ea = float(np.max(np.abs(got["alpha"] - a_star)))
    eb = float(np.max(np.abs(got["beta"] - b_star)))
    ed = float(np.max(np.abs(got["alpha"] - det["alpha"])))
    r1, r2 = _recon(got, G1, G2)
    _say(f"   vs oracle {e}; vs planted |da|={ea:.1e} |db|={eb:.1e}; vs deterministic |da|={ed:.1e};"
         f" reconstruction {r1:.1e} {r2:.1e}; flags {_flags(got)} info {got['info'].tolist()}")
    assert got["alpha"].shape == (n,)
    assert max(e.values()) <= 1e-10
    assert ea <= 1e-10 and eb <= 1e-10 and ed <= 1e-10
    assert r1 <= 1e-12 and r2 <= 1e-12
    # alpha = 1 pairs (G2 has rank below n) have beta = 0: zero V columns, flagged
    assert np.sum(got["beta"] < 1e-14) >= 1
    _beta_zero_consistent(got)


@pytest.mark.parametrize("m,p,n,frac2,b", [
    (400, 330, 150, 0.6, 100),    # the paper's block size: one block past each rank, l1 = l2
    (360, 300, 120, 0.45, 16),    # unequal ranks: l1 > l2
])
def test_full_mode_adaptive_gmp(dev, m, p, n, frac2, b):
    """The paper's regime: Algorithm 1 (blocks of b, absolute eps) on both
    matrices of an exactly low-rank GMP from the Sec. 4 generator, then
    Algorithm 2 with t = n, against the oracle's Algorithm 1 + Algorithm 2,
    the deterministic GSVD (Q1 = I, Q2 = I) and the planted alphas."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    G1, G2, a_star, b_star = I.planted_gmp(m, p, n, seed=41 + n, frac=0.6, frac2=frac2)
    eps = 1e-6 * min(np.linalg.norm(G1), np.linalg.norm(G2))
    _say(f"adaptive full mode: planted GMP {m}/{p}x{n}, ranks {round(0.6 * n)}/{round(frac2 * n)}, b={b}")
    g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
    r = R.rgsvd(g1, g2, 1, 0, 0, 9, precision="fp64", mode="full", sizing="adaptive", tol=float(eps), block=b)
    torch.cuda.synchronize()
    got = {kk: v.cpu().numpy() for kk, v in r.items()}
    Q1, _ = O.basis_adaptive(G1, eps, b, 9, 1)
    Q2, _ = O.basis_adaptive(G2, eps, b, 9, 2)
    ref = O.finish(G1, G2, Q1, Q2, n)
    det = O.full_gsvd(G1, G2)
    e = _gsv_err(got, ref)
    ea = float(np.max(np.abs(got["alpha"] - a_star)))
    ed = float(np.max(np.abs(got["alpha"] - det["alpha"])))
    r1, r2 = _recon(got, G1, G2)
    _say(f"   widths gpu {got['info'][1:3].tolist()} oracle {[Q1.shape[1], Q2.shape[1]]}; vs oracle {e}; "
         f"vs planted {ea:.1e}; vs deterministic {ed:.1e}; reconstruction {r1:.1e} {r2:.1e}")
    assert got["info"][1:3].tolist() == [Q1.shape[1], Q2.shape[1]]
    assert got["alpha"].shape == (n,)
    assert max(e.values()) <= 1e-10
    assert ea <= 1e-10 and ed <= 1e-10
    assert r1 <= 1e-12 and r2 <= 1e-12
    _beta_zero_consistent(got)


def test_disjoint_row_supports(dev):
    """G1 lives on columns [0, 40), G2 on [40, 100): the pairs are (1, 0) for
    G1's directions and (0, 1) for G2's.  The spectra are set so that the top
    t = 30 joint directions are G1's 20 and G2's leading 10 (a 1e3 gap)."""
    from oracle import rgsvd as O
    rng = np.random.default_rng(61)
    m, p, n, a = 300, 250, 100, 40

    def part(rows, cols, s):
        U = np.linalg.qr(rng.standard_normal((rows, len(s))))[0]
        Z = np.linalg.qr(rng.standard_normal((cols, len(s))))[0]
        return (U * s) @ Z.T

    G1 = np.zeros((m, n))
    G2 = np.zeros((p, n))
    G1[:, :a] = part(m, a, np.linspace(2.0, 1.0, 20))
    G2[:, a:] = part(p, n - a, np.concatenate([np.linspace(1.9, 1.1, 10), 1e-3 * np.linspace(1, 0.5, 10)]))
    k, o = 30, 10
    _say(f"disjoint supports {m}/{p}x{n}: t={k}")
    got = _run(dev, G1, G2, k, o, 1, 23)
    ref = O.rgsvd(G1, G2, k, o, 1, 23)
    e = _gsv_err(got, ref)
    _say(f"   vs oracle {e}; alpha {np.round(got['alpha'], 12).tolist()[:3]}...; flags {_flags(got)}")
    assert max(e.values()) <= 1e-10
    assert np.allclose(got["alpha"], np.r_[np.ones(20), np.zeros(10)], atol=1e-10)
    assert np.allclose(got["theta"], np.r_[np.full(20, np.pi / 4), np.full(10, -np.pi / 4)], atol=1e-10)
    r1, r2 = _recon(got, G1, G2)
    assert r1 <= 1e-12 and r2 <= 1e-3   # G2's 1e-3 tail lies outside the t = 30 directions
    _beta_zero_consistent(got)
    assert "beta_zero" in _flags(got)


def test_scaled_pair_cluster(dev):
    """G1 = c G2 (c = 1/2): every alpha equals c / sqrt(1 + c^2), theta =
    arctan(c) - pi/4 and D1 = D2 = 1 (uniform P over the t pairs)."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    c, k = 0.5, 10
    j = np.arange(15)
    s = np.where(j < k, 0.9 ** j, 1e-3 * 0.8 ** j)
    _, G2 = I.lowrank_pair(400, 400, 120, 15, s, s, 71)
    G1 = c * G2
    _say(f"scaled pair G1 = {c} G2, 400x120, t={k}")
    got = _run(dev, G1, G2, k, 10, 1, 29)
    ref = O.rgsvd(G1, G2, k, 10, 1, 29)
    e = _gsv_err(got, ref)
    a0 = c / np.sqrt(1 + c * c)
    _say(f"   vs oracle {e}; max|alpha - c/sqrt(1+c^2)| {np.max(np.abs(got['alpha'] - a0)):.1e}; D {got['D']}")
    assert max(e.values()) <= 1e-10
    assert np.max(np.abs(got["alpha"] - a0)) <= 1e-12
    assert np.max(np.abs(got["theta"] - (np.arctan(c) - np.pi / 4))) <= 1e-12
    assert np.max(np.abs(got["D"] - 1.0)) <= 1e-12
    r1, r2 = _recon(got, G1, G2)
    assert r1 <= 1e-2 and r2 <= 1e-2   # the 1e-3 tail of the spectrum is outside t


def test_rank_deficient_sketch_shift_flag(dev):
    """G1 and G2 of exact rank 6 (shared row space) with l = 20: the sketches'
    Grams are singular, so CholeskyQR shifts (flag shift_y) and the extra basis
    vectors carry only rounding.  The t = 4 dominant pairs are gap-separated
    (joint singular values 1.22, 1, 0.81, 0.68, then 1.4e-3) and equal
    s1_j / sqrt(s1_j^2 + s2_j^2): against the oracle (whose Householder QR
    completes the basis with rounding directions too) and that closed form."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    j = np.arange(6)
    s1 = np.where(j < 4, 0.8 ** j, 1e-3)
    s2 = np.array([0.7, 0.6, 0.5, 0.45, 1e-3, 1e-3])
    G1, G2 = I.lowrank_pair(500, 400, 200, 6, s1, s2, 91)
    got = _run(dev, G1, G2, 4, 16, 1, 31)
    ref = O.rgsvd(G1, G2, 4, 16, 1, 31)
    e = _gsv_err(got, ref)
    closed = (s1 / np.sqrt(s1 ** 2 + s2 ** 2))[:4]
    ec = float(np.max(np.abs(got["alpha"] - closed)))
    _say(f"rank-6 pair, l=20: vs oracle {e}; vs closed form {ec:.1e}; flags {_flags(got)} info {got['info'].tolist()}")
    assert "shift_y" in _flags(got)
    assert e["alpha"] <= 1e-8 and e["beta"] <= 1e-8 and e["theta"] <= 1e-8 and ec <= 1e-8
    assert np.max(np.abs(got["alpha"] ** 2 + got["beta"] ** 2 - 1)) <= 1e-12


def test_nonfinite_input_flagged(dev):
    from paper_2404_09459_amd import inputs as I
    G1, G2 = I.small_fp64_pair()["G1"].copy(), I.small_fp64_pair()["G2"]
    G1[17, 33] = np.nan
    _say("NaN in G1[17, 33]: the run must end with FLAG_NONFINITE")
    got = _run(dev, G1, G2, 20, 10, 1, 1)
    _say(f"   flags {_flags(got)} info {got['info'].tolist()} alpha[:3] {got['alpha'][:3]}")
    assert "nonfinite" in _flags(got)
    assert np.all(np.isnan(got["alpha"])) and np.all(np.isnan(got["D"]))
    # a clean run on the same plan afterwards is unaffected
    clean = _run(dev, I.small_fp64_pair()["G1"], G2, 20, 10, 1, 1)
    assert "nonfinite" not in _flags(clean) and np.all(np.isfinite(clean["alpha"]))


def test_nonfinite_input_flagged_staged(dev):
    """The same at t = 120, where H's eigenproblem runs on the block Jacobi and
    H = L1^T L1 and L Y on multi-workgroup launches between the small step's
    stages: NaN GSVs and the flag, and a clean run on the same plan before and
    after gives bit-identical results (no state left behind)."""
    from paper_2404_09459_amd import inputs as I
    m, p, n, k = 1200, 1000, 400, 120
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.95 ** j, 77, noise_entry=1e-6, dtype=np.float64)
    before = _run(dev, G1, G2, k, 10, 1, 3)
    assert "nonfinite" not in _flags(before) and np.all(np.isfinite(before["alpha"]))
    G1n = G1.copy()
    G1n[5, 7] = np.inf
    _say(f"inf in G1[5, 7] at m={m} p={p} n={n} k={k}: the run must end with FLAG_NONFINITE")
    got = _run(dev, G1n, G2, k, 10, 1, 3)
    _say(f"   flags {_flags(got)} info {got['info'].tolist()}")
    assert "nonfinite" in _flags(got)
    assert np.all(np.isnan(got["alpha"])) and np.all(np.isnan(got["D"]))
    after = _run(dev, G1, G2, k, 10, 1, 3)
    for key in ("alpha", "beta", "theta", "U", "V", "R"):
        assert np.array_equal(before[key], after[key]), key


@pytest.mark.parametrize("m,p,n,k,o,precision", [
    (1200, 1000, 400, 120, 10, "fp64"),    # M's factor order 260 (blocks of 8), H's 120: both on the block Jacobi
    (2000, 1600, 600, 100, 20, "mixed"),   # M's factor order 240 (blocks of 16)
])
def test_jacobi_sweep_launches_match_round_launches(dev, m, p, n, k, o, precision):
    """The block Jacobi's one-launch sweeps (a barrier between rounds; every
    sweep, or the default's last three) turn the same pairs in the same order
    as one launch per round: every output bit-identical, on two runs in a row
    of each plan (the barrier counter starts again with each run)."""
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.96 ** j, 91, noise_entry=1e-6, dtype=np.float64)
    dt = R.F64 if precision == "fp64" else R.F32
    npdt = np.float64 if precision == "fp64" else np.float32
    g1 = torch.from_numpy(np.ascontiguousarray(G1.astype(npdt))).to(dev)
    g2 = torch.from_numpy(np.ascontiguousarray(G2.astype(npdt))).to(dev)
    res, counts = {}, {}
    for name, opt in (("sweep", R.OPT_JACOBI_SWEEPS), ("round", R.OPT_JACOBI_ROUNDS), ("default", 0)):
        _say(f"block Jacobi launches per {name}: m={m} p={p} n={n} k={k} o={o} {precision}")
        plan = R.Plan(R.make_desc(m, p, n, k, o, 2, 5, dt, precision, options=opt), dev)
        runs = []
        for rep in range(2):
            R.lib().rgsvd_profile(plan.h, 1 if rep == 1 else 0)
            out = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev)
            R.run(plan, g1, g2, out)
            torch.cuda.synchronize()
            runs.append({kk: v.cpu().numpy() for kk, v in out.items()})
        counts[name] = sum(1 for tg, _ in R.profile_read(plan) if tg == "bjacobi")
        for key in runs[0]:
            assert np.array_equal(runs[0][key], runs[1][key], equal_nan=True), (name, key)
        res[name] = runs[0]
        _say(f"   info {runs[0]['info'].tolist()} block Jacobi launches {counts[name]}")
    assert "jacobi_m" not in _flags(res["sweep"]) and int(res["sweep"]["info"][5]) >= 2
    assert counts["sweep"] < counts["default"] < counts["round"]
    for name in ("sweep", "default"):
        for key in res["round"]:
            assert np.array_equal(res[name][key], res["round"][key], equal_nan=True), (name, key)


def test_jacobi_sweep_barrier_gives_up_and_flags(dev):
    """The failure path of the one-launch sweeps, forced from the host: with
    the barrier told to give up at its first poll, every workgroup leaves the
    launch at once (no wait left behind), the Jacobi of both factors ends
    there, and the pair carries the sweep-limit flags with finite outputs."""
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    m, p, n, k, o = 1200, 1000, 400, 120, 10
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.96 ** j, 91, noise_entry=1e-6, dtype=np.float64)
    g1 = torch.from_numpy(np.ascontiguousarray(G1)).to(dev)
    g2 = torch.from_numpy(np.ascontiguousarray(G2)).to(dev)
    _say(f"barrier gives up at once: m={m} p={p} n={n} k={k} o={o} fp64, every sweep one launch")
    plan = R.Plan(R.make_desc(m, p, n, k, o, 2, 5, R.F64, "fp64",
                              options=R.OPT_JACOBI_SWEEPS | R.OPT_JACOBI_NOWAIT), dev)
    for rep in range(2):
        out = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev)
        R.run(plan, g1, g2, out)
        torch.cuda.synchronize()
        got = {kk: v.cpu().numpy() for kk, v in out.items()}
        _say(f"   run {rep}: flags {_flags(got)} info {got['info'].tolist()}")
        assert "jacobi_m" in _flags(got) and "jacobi_l1" in _flags(got)
        assert int(got["info"][5]) > 40 and int(got["info"][6]) > 40
        for key in ("alpha", "beta", "theta"):
            assert np.all(np.isfinite(got[key])), key
