"""Learned sizing on the GPU, through the C ABI.

* The network's HIP forward, backward and Adam kernels (FP32) against the
  FP64 oracle of the same network: 1e-5 relative.
* The probe features (16-column probe sketch, FP64 Gram eigenvalues) against
  the oracle's SVD of the same probe: 1e-6 in log10 units where the oracle is
  above -6, the floor region below.
* A learned run uses exactly the (l, q) that the attached network picks from
  the probe features, and reproduces a fixed run at that size (to rounding:
  its buffers are laid out for the largest size).
* Gain: a network trained on GPU-labelled pairs, evaluated on held-out
  pairs, against the method without it (fixed sizes).
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


def test_mlp_kernels_match_oracle(dev):
    from oracle import mlp as M
    from paper_2404_09459_amd import sizing as S
    rng = np.random.default_rng(11)
    params = S.init_params(5, dev)
    B = 37
    X = torch.tensor(rng.uniform(-6, 0, (B, 32)), dtype=torch.float32, device=dev)
    T = torch.tensor(rng.normal(0, 1, (B, 2)), dtype=torch.float32, device=dev)
    Y, act = S.mlp_forward(params, X)
    g, loss = S.mlp_backward(params, X, T, act)
    torch.cuda.synchronize()
    th = params.double().cpu().numpy()
    Xh, Th = X.double().cpu().numpy(), T.double().cpu().numpy()
    Yr, _ = M.forward(th, Xh)
    gr = M.grad(th, Xh, Th)
    ey = np.max(np.abs(Y.cpu().numpy() - Yr)) / np.max(np.abs(Yr))
    eg = np.linalg.norm(g.double().cpu().numpy() - gr) / np.linalg.norm(gr)
    el = abs(float(loss.item()) - M.loss(th, Xh, Th)) / M.loss(th, Xh, Th)
    _say(f"mlp: forward rel {ey:.2e}, gradient rel {eg:.2e}, loss rel {el:.2e}")
    assert ey <= 1e-5 and eg <= 1e-5 and el <= 1e-5
    # one Adam step from zero moments
    mom = torch.zeros_like(params)
    vel = torch.zeros_like(params)
    S.adam(params, g, mom, vel, 1, lr=1e-2)
    torch.cuda.synchronize()
    th2, m2, v2 = M.adam_step(th, g.double().cpu().numpy(), np.zeros_like(th), np.zeros_like(th), 1, 1e-2)
    ea = np.max(np.abs(params.double().cpu().numpy() - th2))
    _say(f"adam: max abs difference {ea:.2e}")
    assert ea <= 1e-6


def test_probe_features_match_oracle(dev):
    from oracle.sizing import features
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import sizing as S
    j = np.arange(30)
    G1, G2 = I.lowrank_pair(1200, 900, 300, 30, 0.7 ** j, 0.85 ** j, 77, noise_spectral=1e-6)
    f = S.probe_features(torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev), 3).cpu().numpy()
    ref = features(G1, G2, 3)
    live = ref > -6
    e = np.max(np.abs(f[live] - ref[live]))
    _say(f"features: {int(live.sum())} live, max |diff| {e:.2e}; gpu {np.round(f, 3).tolist()}")
    assert e <= 1e-6
    assert np.all(f[~live] <= -5.0)


def test_learned_run_uses_network_choice(dev):
    from oracle import mlp as M
    from paper_2404_09459_amd import rgsvd as R
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import sizing as S
    j = np.arange(40)
    G1, G2 = I.lowrank_pair(2000, 1500, 400, 40, 0.9 ** j, 0.8 ** j, 78, noise_spectral=1e-5, dtype=np.float32)
    g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
    k, seed = 20, 4
    params = S.init_params(9, dev)
    plan = R.Plan(R.make_desc(2000, 1500, 400, k, 0, 0, seed, R.F32, "fp64", "learned"), dev)
    R.check(R.lib().rgsvd_set_sizing_model(plan.h, R._ptr(params), R._stream(dev)), "set model")
    o = R.alloc_outputs(plan.t, 2000, 1500, 400, plan.l1 + plan.l2, dev)
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    info = o["info"].cpu().numpy()
    feat = S.probe_features(g1, g2, seed, precision="fp64").double().cpu().numpy()
    y, _ = M.forward(params.double().cpu().numpy(), feat[None, :])
    l, q = S.decide(y[0], k, min(plan.l1, plan.l2))
    _say(f"learned run: network output {np.round(y[0], 3).tolist()} -> (l, q) = ({l}, {q}); info {info.tolist()}")
    assert (info[1], info[2], info[3]) == (l, l, q)
    # the learned plan's buffers are laid out for its capacity (other
    # reduction chunking), so equality is to rounding
    fixed = R.rgsvd(g1, g2, k, l - k, q, seed, precision="fp64")
    torch.cuda.synchronize()
    for key in ("alpha", "beta", "theta", "D"):
        assert np.max(np.abs(o[key].cpu().numpy() - fixed[key].cpu().numpy())) <= 1e-12, key


def test_trained_network_gain(dev):
    """Train on GPU-labelled pairs, evaluate on held-out pairs: the learned
    sizes must keep the angular tolerance on at least 90% of 64 held-out
    pairs at a lower cost (passes over G) than the safe fixed setting
    (2k, q = 3), and pass more often than the cheap fixed default
    (k + 10, q = 2) or at lower cost.  The label margin, the training-set
    size and the rounding of q were settled on pairs of another seed; these
    pairs are fresh draws."""
    from paper_2404_09459_amd import sizing as S
    specs = S.pair_specs(224, seed=21)
    train_specs, test_specs = specs[:160], specs[160:]
    X, T, kept = [], [], []
    for s in train_specs:
        G1, G2 = S.make_pair(s)
        g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
        l, q, _, _ = S.label(g1, g2, s)
        X.append(S.probe_features(g1, g2, 1, precision="mixed").cpu().numpy())
        T.append(S.targets(s["k"], l, q))
    X = torch.tensor(np.array(X), dtype=torch.float32, device=dev)
    T = torch.tensor(np.array(T), dtype=torch.float32, device=dev)
    qs = T[:, 1].cpu().numpy()
    _say(f"labels: q histogram {np.bincount(qs.astype(int), minlength=4).tolist()},"
         f" mean log2(l/k) {float(T[:, 0].mean()):.2f}")
    params, losses = S.train(X, T, dev, epochs=600, lr=3e-3, seed=2)
    _say(f"training loss {[round(x, 4) for x in losses]}")
    assert losses[-1] < 0.5 * losses[0]
    rows = []
    for s in test_specs:
        G1, G2 = S.make_pair(s)
        g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
        k = s["k"]
        cap = min(s["m"], s["p"], s["n"], 224)
        ref = S._run(g1, g2, k, min(2 * k + 50, cap), 4, 1, "fp64")
        idx = S._pinned(ref, k, s["nu"])
        f = S.probe_features(g1, g2, 1, precision="mixed")
        y, _ = S.mlp_forward(params, f[None, :])
        l, q = S.decide(y[0].cpu().numpy(), k, cap)
        res = {}
        for name, (ll, qq) in {"learned": (l, q), "fixed_default": (min(k + 10, cap), 2),
                               "fixed_safe": (min(2 * k, cap), 3)}.items():
            got = S._run(g1, g2, k, ll, qq, 1, "mixed")
            res[name] = (S.passes(got, ref, idx), S.cost(s, ll, qq))
        rows.append(res)
    summ = {name: (np.mean([r[name][0] for r in rows]), np.mean([r[name][1] for r in rows]))
            for name in rows[0]}
    for name, (rate, c) in summ.items():
        _say(f"  {name:14s}: pass rate {rate:.3f}, mean passes over G {c:.2f}")
    lr_, lc = summ["learned"]
    sr, sc = summ["fixed_safe"]
    dr, dc = summ["fixed_default"]
    assert lr_ >= 0.9
    assert lc < sc
    assert lr_ >= dr or lc < dc
