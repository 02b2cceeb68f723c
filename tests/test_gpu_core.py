"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances: the FP64 path matches the FP64 oracle (same Omega) to 1e-10 on
every alpha and beta (alpha^2 + beta^2 = 1, so absolute); quantities to 1e-10;
U, V, R to 1e-8 after per-column sign alignment (the sign convention is
tested separately).
"""
import ctypes
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


# ----------------------------------------------------------- lane layout ---
OUT_ROW = {0: lambda g, i: 4 * i + g, 1: lambda g, i: 4 * g + i, 2: lambda g, i: 4 * g + i}


@pytest.mark.parametrize("which", [0, 1, 2])
def test_mfma_raw_lane_map(dev, which):
    """Each output register of each lane lands where the kernels assume."""
    from paper_2404_09459_amd import rgsvd as R
    rng = np.random.default_rng(10 + which)
    K = 4 if which < 2 else 32
    A = np.round(rng.standard_normal((16, K)) * 8) / 8
    B = np.round(rng.standard_normal((K, 16)) * 8) / 8
    dt = torch.float64 if which == 0 else torch.float32
    At, Bt = torch.tensor(A, dtype=dt, device=dev), torch.tensor(B, dtype=dt, device=dev)
    D = torch.zeros(256, dtype=dt, device=dev)
    R.check(R.lib().rgsvd_selftest_mfma(8 + which, At.data_ptr(), Bt.data_ptr(), D.data_ptr(), None), "raw")
    torch.cuda.synchronize()
    raw = D.cpu().numpy().reshape(64, 4)
    ref = A @ B
    found = {}
    for ln in range(64):
        for i in range(4):
            pos = np.argwhere(np.abs(ref - raw[ln, i]) < 1e-3)
            found[(ln, i)] = [tuple(x) for x in pos]
    bad = [(ln, i, found[(ln, i)]) for ln in range(64) for i in range(4)
           if (OUT_ROW[which](ln // 16, i), ln % 16) not in found[(ln, i)]]
    _say(f"raw lane map which={which}: mismatches {len(bad)}; first {bad[:6]}")
    assert not bad


@pytest.mark.parametrize("which", [0, 1, 2])
def test_mfma_lane_layout(dev, which):
    from paper_2404_09459_amd import rgsvd as R
    _say(f"selftest mfma which={which}")
    rng = np.random.default_rng(which)
    K = 4 if which < 2 else 32
    A = rng.standard_normal((16, K))
    B = rng.standard_normal((K, 16))
    if which == 0:
        At, Bt = torch.tensor(A, device=dev), torch.tensor(B, device=dev)
        D = torch.zeros((16, 16), dtype=torch.float64, device=dev)
        ref, tol = A @ B, 1e-14
    else:
        if which == 2:   # exact in bf16
            A = np.round(A * 8) / 8
            B = np.round(B * 8) / 8
        At = torch.tensor(A, dtype=torch.float32, device=dev)
        Bt = torch.tensor(B, dtype=torch.float32, device=dev)
        D = torch.zeros((16, 16), dtype=torch.float32, device=dev)
        ref, tol = A @ B, 1e-5
    R.check(R.lib().rgsvd_selftest_mfma(which, At.data_ptr(), Bt.data_ptr(), D.data_ptr(), None), "selftest")
    torch.cuda.synchronize()
    assert np.max(np.abs(D.cpu().numpy() - ref)) < tol


# -------------------------------------------------------------- generator ---
@pytest.mark.parametrize("seed,stream,rows,col0,ncols",
                         [(1, 1, 37, 0, 30), ((5 << 32) | 77, 2, 300, 3, 17), (2024, 1, 5, 16, 64)])
def test_philox_words_bit_exact(dev, seed, stream, rows, col0, ncols):
    from paper_2404_09459_amd import rgsvd as R
    from oracle.philox import raw_bits
    _say(f"philox words seed={seed} stream={stream} rows={rows} cols={col0}+{ncols}")
    out = torch.zeros((rows, ncols), dtype=torch.int32, device=dev)
    R.check(R.lib().rgsvd_philox_words(seed, stream, rows, col0, ncols, out.data_ptr(), ncols, None), "words")
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, raw_bits(seed, stream, rows, col0, ncols))


def test_gaussian_fp64_and_fp32(dev):
    from paper_2404_09459_amd import rgsvd as R
    from oracle.philox import gaussian_matrix
    rows, col0, ncols = 513, 5, 43
    ref = gaussian_matrix(99, 1, rows, col0, ncols)
    o64 = torch.zeros((rows, ncols), dtype=torch.float64, device=dev)
    o32 = torch.zeros((rows, ncols), dtype=torch.float32, device=dev)
    R.check(R.lib().rgsvd_gaussian(99, 1, rows, col0, ncols, 0, o64.data_ptr(), ncols, None), "g64")
    R.check(R.lib().rgsvd_gaussian(99, 1, rows, col0, ncols, 1, o32.data_ptr(), ncols, None), "g32")
    torch.cuda.synchronize()
    g64 = o64.cpu().numpy()
    # within a few ulp of the FP64 reference evaluation
    assert np.all(np.abs(g64 - ref) <= 8 * np.spacing(np.abs(ref)) + 1e-15)
    assert np.max(np.abs(o32.cpu().numpy() - ref)) < 5e-5


# -------------------------------------------------------------- parity -----
def _run(dev, G1, G2, k, o, q, seed, precision="fp64", mode="truncated"):
    from paper_2404_09459_amd import rgsvd as R
    g1 = torch.from_numpy(G1).to(dev)
    g2 = torch.from_numpy(G2).to(dev)
    r = R.rgsvd(g1, g2, k, o, q, seed, precision=precision, mode=mode)
    torch.cuda.synchronize()
    return {kk: v.cpu().numpy() if hasattr(v, "cpu") else v for kk, v in r.items()}


def _align(A, B):
    """Flip columns of A to best match B (sign ambiguity)."""
    s = np.sign(np.sum(A * B, axis=0))
    s[s == 0] = 1
    return A * s


def _check_pair(got, ref, tol_gsv=1e-10, tol_vec=1e-8, vecs=True):
    t = len(ref["alpha"])
    assert got["alpha"].shape == (t,)
    da = np.max(np.abs(got["alpha"] - ref["alpha"]))
    db = np.max(np.abs(got["beta"] - ref["beta"]))
    dth = np.max(np.abs(got["theta"] - ref["theta"]))
    dp1 = np.max(np.abs(got["P1"] - ref["P1"]))
    dp2 = np.max(np.abs(got["P2"] - ref["P2"]))
    dd = np.max(np.abs(got["D"] - [ref["D1"], ref["D2"]]))
    _say(f"   |da|={da:.2e} |db|={db:.2e} |dtheta|={dth:.2e} |dP|={max(dp1, dp2):.2e} |dD|={dd:.2e}"
         f" info={got['info'].tolist()}")
    assert da <= tol_gsv and db <= tol_gsv
    assert dth <= tol_gsv and dp1 <= tol_gsv and dp2 <= tol_gsv and dd <= tol_gsv
    # the t dominant singular values of the stacked compressed pair; the tail
    # entries only carry the tail's Frobenius norm, formed as ||B||_F^2 minus
    # the sum of the t leading squares, so its square is known to a rounding
    # multiple of N * eps * ||B||_F^2 (absolute)
    sB, rB = got["sigma_B"], ref["sigma_B"]
    assert np.max(np.abs(sB[:t] - rB[:t])) <= 1e-9 * rB[0]
    fro2 = float(np.sum(rB ** 2))
    tail_err = abs(np.sum(sB[t:] ** 2) - np.sum(rB[t:] ** 2))
    assert tail_err <= 64 * len(rB) * np.finfo(np.float64).eps * fro2
    if vecs:
        U = _align(got["U"], ref["U"])
        V = _align(got["V"], ref["V"])
        Rm = _align(got["R"].T, ref["R"].T).T
        eu = np.max(np.abs(U - ref["U"]))
        ev = np.max(np.abs(V - ref["V"]))
        er = np.max(np.abs(Rm - ref["R"])) / np.max(np.abs(ref["R"]))
        _say(f"   |dU|={eu:.2e} |dV|={ev:.2e} |dR|/|R|={er:.2e}")
        assert eu <= tol_vec and ev <= tol_vec and er <= tol_vec


def test_small_pair_fp64_parity(dev):
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    w = I.small_fp64_pair()
    _say(f"parity {w['name']} fp64")
    got = _run(dev, w["G1"], w["G2"], w["k"], w["oversample"], w["q"], w["seed"])
    ref = O.rgsvd(w["G1"], w["G2"], w["k"], w["oversample"], w["q"], w["seed"])
    _check_pair(got, ref)
    # sign convention: largest-magnitude entry of each row of R positive
    Rg = got["R"]
    assert np.all(Rg[np.arange(Rg.shape[0]), np.argmax(np.abs(Rg), axis=1)] > 0)
    assert got["info"][1] == 30 and got["info"][2] == 30 and got["info"][3] == 1


@pytest.mark.parametrize("m,p,n,k,o,q,dt", [
    (333, 257, 171, 9, 7, 0, np.float64),
    (333, 257, 171, 9, 7, 2, np.float64),
    (700, 1290, 95, 30, 18, 1, np.float64),    # l = 48: three tiles
    (2049, 1500, 300, 40, 10, 1, np.float32),  # fp32 storage, fp64 arithmetic
    (129, 65, 64, 1, 1, 1, np.float64),        # k = 1, l = 2
    (900, 700, 300, 60, 10, 1, np.float64),    # l1 + l2 = 140: the block Jacobi, its ninth block partial
])
def test_ragged_fp64_parity(dev, m, p, n, k, o, q, dt):
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    _say(f"parity m={m} p={p} n={n} k={k} o={o} q={q} dtype={dt.__name__}")
    r = min(2 * k + 5, n, m, p)
    j = np.arange(r)
    G1, G2 = I.lowrank_pair(m, p, n, r, 0.85 ** j, 0.75 ** j, 7 + m, noise_entry=1e-7, dtype=dt)
    got = _run(dev, G1, G2, k, o, q, 11)
    ref = O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), k, o, q, 11)
    _check_pair(got, ref, vecs=(k > 1))


@pytest.mark.parametrize("m,p,n,k,o,q,dt", [
    (3000, 2500, 800, 100, 10, 2, np.float32),  # l1 + l2 = 220, as in the 20000/15000 x 5000 workload
    (2000, 1800, 600, 200, 20, 1, np.float64),  # l1 + l2 = 440
])
def test_gap_separated_parity(dev, m, p, n, k, o, q, dt):
    """Shared rank exactly k over a 1e-7 noise floor: the top-k subspace of the
    stacked compressed pair is well separated, so the GSVs are pinned to 1e-10."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    _say(f"gap parity m={m} p={p} n={n} k={k} o={o} q={q} dtype={dt.__name__}")
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.96 ** j, 5 + n, noise_entry=1e-7, dtype=dt)
    got = _run(dev, G1, G2, k, o, q, 13)
    ref = O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), k, o, q, 13)
    _check_pair(got, ref)


def test_rank_deficient_block_jacobi(dev):
    """Exactly rank 40 (no noise) with l1 + l2 = 160: the pivoted Cholesky of M
    stops at rank 40, so the block Jacobi runs on 40 of 160 columns (blocks
    past the rank are empty).  The spectrum drops by 1e-4 after the first k = 30
    components, which pins the top-k subspace: FP64 parity 1e-10."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    k, r = 30, 40
    j = np.arange(r)
    s1 = np.where(j < k, 0.95 ** j, 1e-4 * 0.9 ** (j - k))
    s2 = np.where(j < k, 0.9 ** j, 1e-4 * 0.8 ** (j - k))
    G1, G2 = I.lowrank_pair(900, 800, 300, r, s1, s2, 77)
    _say("parity rank-deficient M: 900/800 x 300, rank 40, k=30, o=50")
    got = _run(dev, G1, G2, k, 50, 1, 5)
    ref = O.rgsvd(G1, G2, k, 50, 1, 5)
    _say(f"   info {got['info'].tolist()}")
    _check_pair(got, ref, vecs=False)


def test_determinism_bitwise(dev):
    from paper_2404_09459_amd import inputs as I
    w = I.small_fp64_pair()
    a = _run(dev, w["G1"], w["G2"], 20, 10, 1, 1)
    b = _run(dev, w["G1"], w["G2"], 20, 10, 1, 1)
    for key in ("alpha", "beta", "theta", "U", "V", "R", "sigma_B"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("m,p,n,k,o,q", [
    (4093, 2711, 517, 150, 10, 1),   # 160-wide basis: the split G^T Q pass runs two waves per column tile
    (3001, 2077, 333, 40, 8, 2),     # 48-wide basis, n = 10 x 32 + 13, ragged row chunks
])
def test_mixed_ragged_gate(dev, m, p, n, k, o, q):
    """The mixed path on ragged shapes (m, p and n off every tile multiple)
    against the FP64 oracle: 1e-4 on the pinned angular distances, the
    GSV pairs on the unit circle."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    _say(f"mixed ragged gate m={m} p={p} n={n} k={k} o={o} q={q}")
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.95 ** j, 7 + n, noise_spectral=1e-5, dtype=np.float32)
    got = _run(dev, G1, G2, k, o, q, 23, precision="mixed")
    ref = O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), k, o, q, 23)
    s = ref["sigma_B"]
    weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
    idx = np.where(weak >= 10 * 1e-5)[0] if s[k - 1] >= 2 * s[k] else np.arange(0)
    dth = np.max(np.abs(got["theta"][idx] - ref["theta"][idx]))
    _say(f"   pinned {len(idx)}/{k} |dtheta|={dth:.2e} info={got['info'].tolist()}")
    assert len(idx) >= k // 2
    assert dth <= 1e-4
    assert np.max(np.abs(got["alpha"] ** 2 + got["beta"] ** 2 - 1)) <= 1e-12


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
def test_reduced_precision_gate(dev, precision):
    """BF16/FP32 sketch paths against the FP64 oracle: 1e-4 on the angular
    distances of the pairs whose weaker component min(alpha_i, beta_i) ||R_i||
    is above the noise floor (the k-subspace being gap-separated), 1e-5 on the
    entropies."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    m, p, n, k, o, q = 3000, 2500, 800, 100, 10, 2
    _say(f"{precision} gate m={m} p={p} n={n} k={k} q={q}")
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.96 ** j, 5 + n, noise_spectral=1e-4,
                            dtype=np.float32)
    got = _run(dev, G1, G2, k, o, q, 21, precision=precision)
    ref = O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), k, o, q, 21)
    s = ref["sigma_B"]
    assert s[k - 1] >= 2 * s[k]
    weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
    idx = np.where(weak >= 10 * 1e-4)[0]
    dth = np.max(np.abs(got["theta"][idx] - ref["theta"][idx]))
    dd = np.max(np.abs(got["D"] - [ref["D1"], ref["D2"]]))
    _say(f"   pinned {len(idx)}/{k} |dtheta|={dth:.2e} (all {np.max(np.abs(got['theta'] - ref['theta'])):.2e})"
         f" |dD|={dd:.2e} info={got['info'].tolist()}")
    assert len(idx) == k
    assert dth <= 1e-4 and dd <= 1e-5
    assert np.max(np.abs(got["alpha"] ** 2 + got["beta"] ** 2 - 1)) <= 1e-12
