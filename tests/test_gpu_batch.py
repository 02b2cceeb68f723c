"""Batched runs: many uneven pairs in one captured graph, through the C ABI.

Each pair of the batch must match the FP64 oracle as a single run does
(FP64 path: 1e-10 on alpha, beta, theta, P, D), every replay of the graph
must reproduce the first one bit for bit (with unrelated eager work and
synchronisations between replays), and the mixed-precision batch must meet
1e-4 on the angular distances of pairs above the noise floor and 1e-5 on the
entropies of pairs whose t pairs all are.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NPAIRS = 12
OVERSAMPLE = 10
Q = 1


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


@pytest.fixture(scope="module")
def batch():
    """Uneven pairs shaped like the 256-pair workload (shared rank 10..30,
    decays 0.6..0.95, per-entry noise 1e-5), scaled down in m, p and n."""
    from paper_2404_09459_amd import inputs as I
    specs = I.batch_specs(npairs=NPAIRS, seed=7, m_range=(300, 3000), n_range=(50, 300),
                          r_range=(10, 30))
    pairs = [I.batch_pair(s, dtype=np.float32) for s in specs]
    return specs, pairs


@pytest.fixture(scope="module")
def refs(batch):
    from oracle import rgsvd as O
    specs, pairs = batch
    return [O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), s["k"], OVERSAMPLE, Q, 1000 + i)
            for i, (s, (G1, G2)) in enumerate(zip(specs, pairs))]


def _plan(dev, specs, precision):
    from paper_2404_09459_amd import rgsvd as R
    descs = [R.make_desc(s["m"], s["p"], s["n"], s["k"], OVERSAMPLE, Q, 1000 + i, R.F32, precision)
             for i, s in enumerate(specs)]
    return R.BatchPlan(descs, dev)


def _host(outs):
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]


def _pinned(ref, k, nu):
    """Indices (in alpha order) of pairs whose weaker component is above the
    noise floor, min(alpha_i, beta_i) ||R_i|| >= 10 nu, taken only when the
    dominant k-subspace of the stacked pair is gap-separated,
    sigma_k(B) >= 2 sigma_{k+1}(B).  Below the floor the angle depends on which
    noise directions the sketch captured, so it is reported, not gated."""
    s = np.asarray(ref["sigma_B"])
    if s[k - 1] < 2 * s[k]:
        return np.arange(0)
    weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
    return np.where(weak >= 10 * nu)[0]


def test_batch_fp64_matches_oracle_and_replays(dev, batch, refs):
    specs, pairs = batch
    _say(f"batch fp64: {NPAIRS} pairs, m,p in [300,3000], n in [50,300]")
    plan = _plan(dev, specs, "fp64")
    dpairs = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in pairs]
    plan.bind(dpairs)
    plan.run()
    torch.cuda.synchronize()
    first = _host(plan.outs)
    for i, (got, ref) in enumerate(zip(first, refs)):
        da = np.max(np.abs(got["alpha"] - ref["alpha"]))
        db = np.max(np.abs(got["beta"] - ref["beta"]))
        dth = np.max(np.abs(got["theta"] - ref["theta"]))
        dp = max(np.max(np.abs(got["P1"] - ref["P1"])), np.max(np.abs(got["P2"] - ref["P2"])))
        dd = np.max(np.abs(got["D"] - [ref["D1"], ref["D2"]]))
        _say(f"  pair {i} m={specs[i]['m']} p={specs[i]['p']} n={specs[i]['n']} k={specs[i]['k']}:"
             f" |da|={da:.1e} |db|={db:.1e} |dtheta|={dth:.1e} |dP|={dp:.1e} |dD|={dd:.1e}"
             f" info={got['info'].tolist()}")
        assert max(da, db, dth, dp, dd) <= 1e-10
        assert got["info"][0] == 0
    # replays with unrelated eager work in between reproduce the first run
    x = torch.randn(512, 512, device=dev)
    for rep in range(3):
        y = (x @ x).sum()
        torch.cuda.synchronize()
        for o in plan.outs:
            for v in o.values():
                v.fill_(float("nan")) if v.is_floating_point() else v.zero_()
        plan.run()
        torch.cuda.synchronize()
        again = _host(plan.outs)
        for a, b in zip(first, again):
            for key in a:
                assert np.array_equal(a[key], b[key], equal_nan=False), (rep, key)
        _say(f"  replay {rep}: identical (eager work {float(y):.3e})")


def test_batch_matches_single_runs(dev, batch):
    from paper_2404_09459_amd import rgsvd as R
    specs, pairs = batch
    plan = _plan(dev, specs[:4], "fp64")
    dpairs = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in pairs[:4]]
    plan.bind(dpairs)
    plan.run()
    torch.cuda.synchronize()
    bat = _host(plan.outs)
    for i, (s, (g1, g2)) in enumerate(zip(specs[:4], dpairs)):
        one = R.rgsvd(g1, g2, s["k"], OVERSAMPLE, Q, 1000 + i)
        torch.cuda.synchronize()
        d = np.max(np.abs(one["alpha"].cpu().numpy() - bat[i]["alpha"]))
        _say(f"  pair {i}: batched vs single |da|={d:.1e}")
        assert d <= 1e-12


def test_batch_mixed_accuracy_gate(dev, batch, refs):
    specs, pairs = batch
    _say(f"batch mixed (bf16 sketch): {NPAIRS} pairs")
    plan = _plan(dev, specs, "mixed")
    dpairs = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in pairs]
    plan.bind(dpairs)
    plan.run()
    torch.cuda.synchronize()
    got = _host(plan.outs)
    full = 0
    for i, (g, ref, s) in enumerate(zip(got, refs, specs)):
        nu = s["noise"] * (np.sqrt(max(s["m"], s["p"])) + np.sqrt(s["n"]))
        idx = _pinned(ref, s["k"], nu)
        dth = np.max(np.abs(g["theta"][idx] - ref["theta"][idx])) if len(idx) else 0.0
        dall = np.max(np.abs(g["theta"] - ref["theta"]))
        dd = np.max(np.abs(g["D"] - [ref["D1"], ref["D2"]]))
        _say(f"  pair {i}: pinned {len(idx)}/{s['k']} |dtheta| pinned {dth:.1e} (all {dall:.1e})"
             f" |dD|={dd:.1e}")
        assert dth <= 1e-4
        if len(idx) == s["k"]:        # entropies sum over all t pairs: gated when all are pinned
            full += 1
            assert dd <= 1e-5
    assert full >= 3


def test_batch_block_jacobi_sizes(dev):
    """A batch whose pairs take both Jacobi paths: l1 + l2 = 60 (one workgroup,
    LDS), 160 (block Jacobi, 16-column blocks) and 300 (block Jacobi, 8-column
    blocks, and t = 140 > 100, so H's factor takes the block Jacobi too).
    Shared rank exactly k over a 1e-7 floor, so every GSV is pinned: FP64
    parity 1e-10 per pair, and bit-identical replays of the captured graph."""
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    cfg = [(700, 600, 200, 20), (1200, 1000, 300, 70), (1500, 1400, 400, 140)]
    specs, pairs, refs = [], [], []
    for i, (m, p, n, k) in enumerate(cfg):
        j = np.arange(k)
        G1, G2 = I.lowrank_pair(m, p, n, k, 0.97 ** j, 0.95 ** j, 31 + i, noise_entry=1e-7)
        specs.append(dict(m=m, p=p, n=n, k=k))
        pairs.append((G1, G2))
        refs.append(O.rgsvd(G1, G2, k, OVERSAMPLE, Q, 2000 + i))
    descs = [R.make_desc(s["m"], s["p"], s["n"], s["k"], OVERSAMPLE, Q, 2000 + i, R.F64, "fp64")
             for i, s in enumerate(specs)]
    plan = R.BatchPlan(descs, dev)
    dpairs = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in pairs]
    plan.bind(dpairs)
    plan.run()
    torch.cuda.synchronize()
    first = _host(plan.outs)
    for i, (got, ref, s) in enumerate(zip(first, refs, specs)):
        da = np.max(np.abs(got["alpha"] - ref["alpha"]))
        db = np.max(np.abs(got["beta"] - ref["beta"]))
        dth = np.max(np.abs(got["theta"] - ref["theta"]))
        dd = np.max(np.abs(got["D"] - [ref["D1"], ref["D2"]]))
        _say(f"  pair {i} l1+l2={2 * (s['k'] + OVERSAMPLE)} k={s['k']}: |da|={da:.1e} |db|={db:.1e}"
             f" |dtheta|={dth:.1e} |dD|={dd:.1e} info={got['info'].tolist()}")
        assert max(da, db, dth, dd) <= 1e-10
        assert got["info"][0] == 0 and got["info"][4] == 0
    for rep in range(2):
        for o in plan.outs:
            for v in o.values():
                v.fill_(float("nan")) if v.is_floating_point() else v.zero_()
        plan.run()
        torch.cuda.synchronize()
        again = _host(plan.outs)
        for a, b in zip(first, again):
            for key in a:
                assert np.array_equal(a[key], b[key]), (rep, key)
