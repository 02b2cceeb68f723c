"""The allocation-free entry point rgsvd_run_static (workspace in the
library's static device scratch) against rgsvd_run (caller's workspace) on
the same plans, through the C ABI: two calls in a row, the second with a
smaller pair and another precision, then the first plan again after the
second has overwritten the scratch.  FP64 runs must agree to 1e-10 (the
FP64 parity bar), the mixed run to 1e-12 (same kernels, same order)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


KEYS = ("alpha", "beta", "theta", "P1", "P2", "D", "sigma_B", "Ut", "Vt", "R")


def _pair(dev, m, p, n, r, seed, dtype):
    from paper_2404_09459_amd import inputs as I
    j = np.arange(r)
    G1, G2 = I.lowrank_pair(m, p, n, r, 0.85 ** j, 0.75 ** j, seed, noise_entry=1e-7, dtype=dtype)
    return torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)


def _both(dev, plan, g1, g2):
    from paper_2404_09459_amd import rgsvd as R
    m, n = g1.shape
    p = g2.shape[0]
    a = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev)
    b = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev)
    R.run_static(plan, g1, g2, a)
    torch.cuda.synchronize()
    R.run(plan, g1, g2, b)
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in a.items()}, {k: v.cpu().numpy() for k, v in b.items()})


def _cmp(a, b, tol):
    worst = max(float(np.max(np.abs(a[k] - b[k]))) for k in KEYS)
    assert a["info"].tolist() == b["info"].tolist()
    assert worst <= tol, worst
    return worst


def test_static_run_matches_workspace_run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_09459_amd import rgsvd as R
    dev = torch.device("cuda:0")
    R.lib()
    g1, g2 = _pair(dev, 1000, 800, 300, 40, 3, np.float64)
    h1, h2 = _pair(dev, 600, 500, 200, 30, 4, np.float32)
    pa = R.Plan(R.make_desc(1000, 800, 300, 20, 10, 1, 7, R.F64, "fp64"), dev)
    pb = R.Plan(R.make_desc(600, 500, 200, 12, 8, 2, 8, R.F32, "mixed"), dev)
    assert pa.ws_bytes <= R.STATIC_SCRATCH_BYTES and pb.ws_bytes < pa.ws_bytes
    _say(f"static run 1: 1000/800x300 fp64 (workspace {pa.ws_bytes / 2**20:.1f} MiB)")
    wa = _cmp(*_both(dev, pa, g1, g2), 1e-10)
    _say(f"static run 2: 600/500x200 mixed (workspace {pb.ws_bytes / 2**20:.1f} MiB)")
    wb = _cmp(*_both(dev, pb, h1, h2), 1e-12)
    _say("static run 3: the first plan again")
    wc = _cmp(*_both(dev, pa, g1, g2), 1e-10)
    _say(f"   max differences {wa:.1e} {wb:.1e} {wc:.1e}")
