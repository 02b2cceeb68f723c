"""Autotuner of the streaming kernels' tile shapes, through the C ABI: the
choice is at least as fast as the heuristic default (it is among the timed
candidates), and the tuned plans keep their accuracy (single pair against
the untuned run; a batch against the FP64 oracle's gap-separated angles)."""
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


def _time(plan, g1, g2, o, reps=5):
    from paper_2404_09459_amd import rgsvd as R
    R.run(plan, g1, g2, o)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        R.run(plan, g1, g2, o)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def test_autotune_single_pair(dev):
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    m, p, n, k, o_, q = 8000, 6000, 2000, 60, 10, 2
    j = np.arange(k)
    G1, G2 = I.lowrank_pair(m, p, n, k, 0.95 ** j, 0.93 ** j, 31, noise_spectral=1e-4, dtype=np.float32)
    g1, g2 = torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)
    plan = R.Plan(R.make_desc(m, p, n, k, o_, q, 9, R.F32, "mixed"), dev)
    out = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev)
    t_default = _time(plan, g1, g2, out)
    base = {key: out[key].cpu().numpy().copy() for key in ("theta", "D")}
    choice, ms = R.autotune(plan, g1, g2, out, reps=2)
    t_tuned = _time(plan, g1, g2, out)
    dth = np.max(np.abs(out["theta"].cpu().numpy() - base["theta"]))
    _say(f"autotune {m}/{p}x{n} l={k + o_}: choice (rt, js, chunk, family) = {choice}, tuner {ms:.3f} ms;"
         f" default {t_default:.3f} ms -> tuned {t_tuned:.3f} ms; |dtheta| vs default {dth:.1e}")
    assert t_tuned <= 1.10 * t_default
    assert dth <= 1e-5
    # a new plan of the same shape starts from the cached choice
    plan2 = R.Plan(R.make_desc(m, p, n, k, o_, q, 9, R.F32, "mixed"), dev)
    out2 = R.alloc_outputs(plan2.t, m, p, n, plan2.l1 + plan2.l2, dev)
    t2 = _time(plan2, g1, g2, out2)
    _say(f"   new plan of the same shape: {t2:.3f} ms")
    assert np.array_equal(out2["theta"].cpu().numpy(), out["theta"].cpu().numpy())


def test_autotune_batch_keeps_accuracy(dev):
    from oracle import rgsvd as O
    from paper_2404_09459_amd import inputs as I
    from paper_2404_09459_amd import rgsvd as R
    specs = I.batch_specs(npairs=8, seed=17, m_range=(1000, 4000), n_range=(80, 300), r_range=(10, 30))
    pairs = [I.batch_pair(s, dtype=np.float32) for s in specs]
    descs = [R.make_desc(s["m"], s["p"], s["n"], s["k"], 10, 2, 50 + i, R.F32, "mixed") for i, s in enumerate(specs)]
    bp = R.BatchPlan(descs, dev)
    dpairs = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in pairs]
    choice, ms = bp.autotune(dpairs, reps=2)
    bp.run()
    torch.cuda.synchronize()
    _say(f"batch autotune: choice {choice}, {ms:.3f} ms per batch")
    worst = 0.0
    for i, (s, (G1, G2), o) in enumerate(zip(specs, pairs, bp.outs)):
        ref = O.rgsvd(G1.astype(np.float64), G2.astype(np.float64), s["k"], 10, 2, 50 + i)
        nu = s["noise"] * (np.sqrt(max(s["m"], s["p"])) + np.sqrt(s["n"]))
        sB = ref["sigma_B"]
        weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
        idx = np.where(weak >= 10 * nu)[0] if sB[s["k"] - 1] >= 2 * sB[s["k"]] else np.arange(0)
        if len(idx):
            worst = max(worst, float(np.max(np.abs(o["theta"].cpu().numpy()[idx] - ref["theta"][idx]))))
    _say(f"   worst pinned |dtheta| over the batch {worst:.1e}")
    assert worst <= 1e-4
