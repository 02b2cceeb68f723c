"""Learned sizing on the GPU, through the C ABI.

* The network's HIP forward, backward and Adam kernels (FP32) against the
  FP64 oracle of the same network: 1e-5 relative.
* The sizing features (16-column probe sketch, FP64 Gram eigenvalues; the
  R-diagonal profile of the widest sketch from its CholeskyQR Cholesky)
  against the oracle's SVD of the same probe and QR of the same sketch.
* A learned run uses exactly the (l, q) that the attached network picks from
  the probe features, and reproduces a fixed run at that size (to rounding:
  its buffers are laid out for the largest size).
* The residual judge accepts a sketch that spans the range and sends one
  that does not to Algorithm 1, whose result equals an adaptive run's.
* Gain: a network trained on GPU-labelled pairs, evaluated on held-out
  pairs against the method without it (fixed sizes) and against the
  adaptive range finder, in measured time; unpinned pairs counted apart.
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
    """FP64 plan against the oracle's SVD of the probe and QR of the widest
    sketch (same Omega columns).  The Gram route resolves a ratio r to about
    eps / r^2 relative: 1e-6 in log10 units on the probe above -6 and on the
    profile above -4, 1e-3 on the profile between -6 and -4, and the floor
    region (oracle below -6) at most -5."""
    from oracle.sizing import features
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import sizing as S
    j = np.arange(30)
    G1, G2 = I.lowrank_pair(1200, 900, 300, 30, 0.7 ** j, 0.85 ** j, 77, noise_spectral=1e-6)
    k = 20
    f = S.probe_features(torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev), 3, k).cpu().numpy()
    ref = features(G1, G2, 3, k, 224)
    probe = np.r_[0:8, 16:24]
    prof = np.r_[8:16, 24:32]
    d = np.abs(f - ref)
    _say(f"features: gpu {np.round(f, 3).tolist()}")
    _say(f"features: oracle {np.round(ref, 3).tolist()}")
    assert np.all(d[probe][ref[probe] > -6] <= 1e-6)
    assert np.all(d[prof][ref[prof] > -4] <= 1e-6)
    assert np.all(d[prof][(ref[prof] > -6) & (ref[prof] <= -4)] <= 1e-3)
    assert np.all(f[ref <= -6] <= -5.0)
    # the profile half is live down to the pair's noise floor
    assert np.sum(ref[prof] > -4) >= 8


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
    feat = S.probe_features(g1, g2, seed, k, precision="fp64").double().cpu().numpy()
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


def _learned_plan(dev, m, p, n, k, seed, params, precision="fp64", tol=0.0, block=0, lmax=0, dt=None):
    from paper_2404_09459_amd import rgsvd as R
    plan = R.Plan(R.make_desc(m, p, n, k, 0, 0, seed, dt if dt is not None else R.F64, precision, "learned",
                              "truncated", tol, block, lmax), dev)
    R.check(R.lib().rgsvd_set_sizing_model(plan.h, R._ptr(params), R._stream(dev)), "set model")
    return plan


def test_residual_judge_accepts_and_falls_back(dev):
    """Exactly rank-40 pair, tol 1e-4.  With k = 36 every grid width (>= 40)
    spans the range and the residual is the cumulative form's rounding floor
    (about 1e-6 here: ||G||_F^2 and ||Q^T G||_F^2 are FP64 sums of 1e5
    squares), so the judge accepts the network's sketch.  With k = 8 and a
    width cap of 24 every grid width is below the rank, the residual is the
    energy of components 24..39 (above 1e-3), and the judge sends the pair
    to Algorithm 1 (b = 16, same tol, same cap), whose result must equal an
    adaptive run's."""
    from paper_2404_09459_amd import rgsvd as R
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import sizing as S
    j = np.arange(40)
    G1, G2 = I.lowrank_pair(800, 700, 200, 40, 0.85 ** j, 0.75 ** j, 47)
    g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
    params = S.init_params(9, dev)
    tol = 1e-4
    plan = _learned_plan(dev, 800, 700, 200, 36, 5, params, tol=tol)
    o = R.alloc_outputs(plan.t, 800, 700, 200, plan.l1 + plan.l2, dev)
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    info = o["info"].cpu().numpy()
    _say(f"judge, k=36: info {info.tolist()} flags {R.decode_flags(int(info[4]))}")
    assert "fallback" not in R.decode_flags(int(info[4])) and info[1] >= 40
    plan = _learned_plan(dev, 800, 700, 200, 8, 5, params, tol=tol, block=16, lmax=24)
    o = R.alloc_outputs(plan.t, 800, 700, 200, plan.l1 + plan.l2, dev)
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    got = {kk: v.cpu().numpy() for kk, v in o.items()}
    ada = R.rgsvd(g1, g2, 8, 0, 0, 5, sizing="adaptive", tol=tol, block=16, lmax=24)
    torch.cuda.synchronize()
    ada = {kk: v.cpu().numpy() for kk, v in ada.items()}
    _say(f"judge, k=8, cap 24: info {got['info'].tolist()} flags {R.decode_flags(int(got['info'][4]))};"
         f" adaptive info {ada['info'].tolist()}")
    assert "fallback" in R.decode_flags(int(got["info"][4]))
    assert got["info"][1:3].tolist() == ada["info"][1:3].tolist() == [24, 24]
    for key in ("alpha", "beta", "theta", "D"):
        assert np.max(np.abs(got[key] - ada[key])) <= 1e-10, key
    # the next call on the same plan starts again from the network's choice
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    assert "fallback" in R.decode_flags(int(o["info"][4].item()))


def _compare(dev, specs, params, make):
    """Pass rate (pinned pairs only) and measured time of the learned run,
    the fixed default (k + 10, q = 2) in mixed precision and in FP64, the
    safe fixed setting (2k, q = 3) and the adaptive range finder
    (Algorithm 1, b = 16, eps = the Frobenius norm of the larger noise
    matrix, FP64) on each pair of specs."""
    from paper_2404_09459_amd import sizing as S
    rows, unpinned = [], 0
    for s in specs:
        g1, g2 = make(s)
        k = s["k"]
        cap = min(s["m"], s["p"], s["n"], 224)
        ref = S._run(g1, g2, k, min(2 * k + 50, cap), 4, 1, "fp64")
        idx = S._pinned(ref, k, s["nu"])
        if len(idx) == 0:
            unpinned += 1
            continue
        res = {}
        got, ms = S._run(g1, g2, k, k, 0, 1, "mixed", timed=True, sizing="learned", model=params)
        res["learned"] = (S.passes(got, ref, idx), ms, int(got["info"][3]))
        for name, (ll, qq) in {"fixed_default": (min(k + 10, cap), 2), "fixed_safe": (min(2 * k, cap), 3)}.items():
            got, ms = S._run(g1, g2, k, ll, qq, 1, "mixed", timed=True)
            res[name] = (S.passes(got, ref, idx), ms, qq)
        got, ms = S._run(g1, g2, k, min(k + 10, cap), 2, 1, "fp64", timed=True)
        res["fp64_default"] = (S.passes(got, ref, idx), ms, 2)
        noise = max(s["nu"] * np.sqrt(rows_ * s["n"]) / (np.sqrt(rows_) + np.sqrt(s["n"]))
                    for rows_ in (s["m"], s["p"]))
        got, ms = S._run(g1, g2, k, k, 0, 1, "fp64", timed=True, sizing="adaptive", tol=float(noise), block=16)
        res["adaptive"] = (S.passes(got, ref, idx), ms, 0)
        rows.append(res)
        del g1, g2
    summ = {name: (float(np.mean([r[name][0] for r in rows])), float(np.mean([r[name][1] for r in rows])))
            for name in rows[0]}
    return summ, len(rows), unpinned


def test_trained_network_gain(dev):
    """Train on GPU-labelled pairs, evaluate on held-out pairs.  A pair with no
    pinned index (no gap at k, or every weaker component below the noise
    floor) has no label and no verdict: it is left out of training and
    counted apart.  The network trains on pairs with the learned-sizing
    workload's ranks on fewer rows (sizing.TRAIN_RANGES: m, p <= 4000) and
    on 24 at the workload's own scale (sizing.TRAIN_LARGE); on held-out
    pairs of the first recipe it must keep the angular tolerance on at
    least 90% of the pinned ones.
    At that scale every run is set by the small step's fixed latency, so
    times are only reported.  The gain is measured on held-out pairs from
    the workload's upper range (m, p in [20000, 50000], n in [1000, 2000]),
    where the passes over G weigh in: there the learned run (mixed
    precision) must pass at least 85% of the pinned pairs and cost less
    measured time than the FP64 run at the fixed default (k + 10, q = 2),
    than the safe fixed setting (2k, q = 3) and than the adaptive range
    finder; against the mixed fixed default it must pass as often or cost
    less.  The label margin, the training-set size and the rounding of q
    were settled on pairs of another seed."""
    from paper_2404_09459_amd import sizing as S
    specs = S.pair_specs(240, seed=21, **S.TRAIN_RANGES)
    train_specs, test_specs = specs[:176], specs[176:]

    def small(s):
        G1, G2 = S.make_pair(s)
        return torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)

    X, T, skipped = S.label_set(dev, train_specs, small)
    X2, T2, skipped2 = S.label_set(dev, S.pair_specs(24, seed=121, **S.TRAIN_LARGE),
                                   lambda s: S.make_pair_device(s, dev))
    X, T, skipped = X + X2, T + T2, skipped + skipped2
    X = torch.tensor(np.array(X), dtype=torch.float32, device=dev)
    T = torch.tensor(np.array(T), dtype=torch.float32, device=dev)
    qs = T[:, 1].cpu().numpy()
    _say(f"labels: {len(X)} pinned training pairs ({skipped} unpinned left out), q histogram "
         f"{np.bincount(qs.astype(int), minlength=4).tolist()}, mean log2(l/k) {float(T[:, 0].mean()):.2f}")
    params, losses = S.train(X, T, dev, epochs=600, lr=3e-3, seed=2)
    _say(f"training loss {[round(x, 4) for x in losses]}")
    assert losses[-1] < 0.5 * losses[0]

    summ, npin, nun = _compare(dev, test_specs, params, small)
    _say(f"held-out, small scale: {npin} pinned pairs, {nun} unpinned counted apart")
    for name, (rate, c) in summ.items():
        _say(f"  {name:14s}: pass rate {rate:.3f}, mean time {c:.3f} ms")
    assert npin >= 20 and summ["learned"][0] >= 0.9

    big_specs = S.pair_specs(40, seed=23, m_range=(20000, 50000), n_range=(1000, 2000), r_range=(5, 100))
    summ, npin, nun = _compare(dev, big_specs, params, lambda s: S.make_pair_device(s, dev))
    _say(f"held-out, large scale: {npin} pinned pairs, {nun} unpinned counted apart")
    for name, (rate, c) in summ.items():
        _say(f"  {name:14s}: pass rate {rate:.3f}, mean time {c:.3f} ms")
    lr_, lt = summ["learned"]
    assert npin >= 5
    assert lr_ >= 0.85
    for base in ("fp64_default", "fixed_safe", "adaptive"):
        assert lt < summ[base][1], base
    br, bt = summ["fixed_default"]
    assert lr_ >= br or lt < bt
