#!/usr/bin/env python3
"""Throughput of the randomized GSVD on one MI355X.

One step = one complete randomized GSVD of a pair (Gaussian sketch, power
iterations with CholeskyQR, projection, the small FP64 GSVD step, recovery of
U, V, R and the comparative quantities), inputs resident in HBM.

Default workload: G1 100000 x 2000, G2 80000 x 2000 FP32, shared rank 200,
decay 0.97 per index, spectral noise floor 1e-3; k = 200, oversampling 20,
two power iterations.  The headline `value` is the mixed-precision path
(BF16 MFMA sketch and first power iteration, FP32 last iteration and
projection, FP64 small step); the FP32 and FP64 paths are timed beside it,
and so is the mixed path with learned sizing (the sizing network trained
first on small pairs that the method labels on the GPU).
Every path is checked against the FP64 CPU oracle run on the same pair with
the same Omega (angular distances within 1e-4 on the gap-separated indices,
entropies within 1e-5).  The literal workload gives G1 and G2 one decay, so
every angular distance sits near zero; the accuracy gate therefore also runs
the mixed path on the same shapes with G2's decay 0.96 (distinct GSVs), again
against the full-size oracle.  The oracle's own time, with all host threads
and with one, is the CPU baseline.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rGSVD pairs/s + sketch TFLOP/s, mixed vs FP64, at angular-dist err<=1e-4"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TF = {"fp64": 78.6, "fp32": 157.3, "mixed": 2516.6}
# 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
FP64_VEC_PEAK_TF = 78.6
# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, each scaled by what it
# reads for a copy kernel of known size (profiles/hbm_counters_*.md), keyed by
# workload: the mixed sketch pass (k_nn, BF16), the block Jacobi launches
# (k_bjinit + k_bjround + k_bjsweep, averaged over the launches of a run) and the small
# step's k_small launches (averaged).  Kernels changed since their counters
# were taken have no entry (traffic null).
TRAFFIC = {"large": {"sketch": 1.659e9, "bjacobi": 2.805e6},
           "medium": {"sketch": 0.743e9, "bjacobi": 0.776e6, "small": 1.397e6}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, distinct=False):
    """(pair, spectral noise floor); distinct=True gives G2 its own decay
    (0.93 medium, 0.96 large) so that the GSVs are spread out."""
    from paper_2404_09459_amd import inputs as I
    if name == "medium":
        return I.medium_fp32_pair(decay2=0.93 if distinct else None), 1e-4
    if name == "small":
        return I.small_fp64_pair(), 1e-6 * (np.sqrt(1000) + np.sqrt(300))
    if name == "large":
        return I.large_fp32_pair(decay2=0.96 if distinct else None), 1e-3
    raise SystemExit(f"unknown workload {name}")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i_.get("num_threads", 1) for i_ in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def time_oracle(G1d, G2d, k, o, q, seed, reps, threads=None):
    """Median wall time of the FP64 oracle on the pair (and its last result);
    threads=1 limits the BLAS/LAPACK pools to one thread."""
    from oracle import rgsvd as O
    from contextlib import nullcontext
    ctx = nullcontext()
    if threads is not None:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=threads)
    times, ref = [], None
    with ctx:
        for r in range(max(1, reps)):
            c0 = time.time()
            ref = O.rgsvd(G1d, G2d, k, o, q, seed)
            times.append(time.time() - c0)
            log(f"[bench] oracle run {r} ({threads or oracle_threads()} threads): {times[-1]:.2f}s")
    return float(np.median(times)), ref


def pinned(ref, t, nu):
    """Indices (alpha order) of pairs whose weaker component is above the
    noise floor, min(alpha_i, beta_i) ||R_i|| >= 10 nu, when the dominant
    t-subspace of the stacked pair is gap-separated (sigma_t >= 2 sigma_{t+1})."""
    s = np.asarray(ref["sigma_B"])
    if len(s) > t and s[t - 1] < 2 * s[t]:
        return np.arange(0)
    weak = np.minimum(ref["alpha"], ref["beta"]) * np.linalg.norm(ref["R"], axis=1)
    return np.where(weak >= 10 * nu)[0]


def errors(got, ref, idx):
    e = dict(alpha=float(np.max(np.abs(got["alpha"] - ref["alpha"]))),
             beta=float(np.max(np.abs(got["beta"] - ref["beta"]))),
             P1=float(np.max(np.abs(got["P1"] - ref["P1"]))),
             P2=float(np.max(np.abs(got["P2"] - ref["P2"]))),
             D=float(np.max(np.abs(got["D"] - np.array([ref["D1"], ref["D2"]])))))
    e["theta_pinned"] = float(np.max(np.abs(got["theta"][idx] - ref["theta"][idx]))) if len(idx) else 0.0
    e["theta_all"] = float(np.max(np.abs(got["theta"] - ref["theta"])))
    e["n_pinned"] = int(len(idx))
    return e


def bench_batch(args):
    """256 uneven pairs (m, p in [2000, 20000], n in [50, 500], shared rank 10..50,
    decays 0.6..0.95, per-entry noise 1e-5, FP32 storage) in one batched plan,
    mixed precision (BF16 sketches), oversample 10 (less where l would exceed
    min(m, p, n)), q = 2, replayed as one captured graph.  The pairs are
    generated on the device from seeded Gaussians: G_i = U_i diag(d_i^j) Z^T +
    noise N_i with U_i, Z orthonormalised.  A sample of pairs is checked
    against the FP64 oracle and timed on the host for the CPU baseline."""
    import torch
    from paper_2404_09459_amd import rgsvd as R
    from paper_2404_09459_amd import inputs as I
    dev = torch.device("cuda:0")
    R.lib()
    specs = I.batch_specs(npairs=256, seed=104)
    q = 2
    t0 = time.time()
    pairs, descs, ovs = [], [], []
    g = torch.Generator(device=dev)
    for i, sp in enumerate(specs):
        g.manual_seed(sp["seed"])
        jj = torch.arange(sp["r"], device=dev, dtype=torch.float64)
        Z = torch.linalg.qr(torch.randn(sp["n"], sp["r"], generator=g, device=dev, dtype=torch.float64))[0]
        mats = []
        for rows, d in ((sp["m"], sp["d1"]), (sp["p"], sp["d2"])):
            U = torch.linalg.qr(torch.randn(rows, sp["r"], generator=g, device=dev, dtype=torch.float64))[0]
            G = (U * (d ** jj)) @ Z.T
            G += sp["noise"] * torch.randn(rows, sp["n"], generator=g, device=dev, dtype=torch.float64)
            mats.append(G.float().contiguous())
        pairs.append((mats[0], mats[1]))
        o = max(0, min(10, sp["n"] - sp["k"], sp["m"] - sp["k"], sp["p"] - sp["k"]))
        ovs.append(o)
        descs.append(R.make_desc(sp["m"], sp["p"], sp["n"], sp["k"], o, q, 5000 + i, R.F32, "mixed"))
    torch.cuda.synchronize()
    log(f"[bench] batch: 256 pairs generated on the device in {time.time() - t0:.1f}s")
    plan = R.BatchPlan(descs, dev)
    tune = None
    if not args.no_tune:
        choice, tms = plan.autotune(pairs, reps=2)
        tune = {"rows_per_tile": choice[0], "cols_per_lane": choice[1],
                "chunks": ["heuristic", "half", "twice"][choice[2]],
                "kernels": {0: None, 1: "8-wave k_nn/k_tn", 2: "per-wave k_gw/k_gtq"}[choice[3]], "ms": tms}
        log(f"[bench] batch: autotuned tile shapes {tune}")
    outs = plan.bind(pairs)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        plan.run()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = len(specs) / (ms * 1e-3)
    log(f"[bench] batch: {ms:.3f} ms per batch of {len(specs)} pairs ({value:.0f} pairs/s)")
    # algorithmic HBM bytes of the streaming passes: 2q + 2 reads of every G
    gbytes = sum((sp["m"] + sp["p"]) * sp["n"] * 4 for sp in specs) * (2 * q + 2)
    roof = {"bound": "hbm", "achieved": gbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
            "kernel": "whole batch graph (every kernel; one replay per step)",
            "avg_launch_ms": ms, "launches_per_step": 1}
    cpu, errs, gate = None, [], None
    if not args.no_cpu:
        from oracle import rgsvd as O
        threads = oracle_threads()
        sample = list(range(0, len(specs), len(specs) // 8))[:8]
        tcpu = 0.0
        worst = 0.0
        for i in sample:
            sp = specs[i]
            G1d = pairs[i][0].double().cpu().numpy()
            G2d = pairs[i][1].double().cpu().numpy()
            c0 = time.time()
            ref = O.rgsvd(G1d, G2d, sp["k"], ovs[i], q, 5000 + i)
            tcpu += time.time() - c0
            got = {kk: v.cpu().numpy() for kk, v in outs[i].items()}
            nu = sp["noise"] * (np.sqrt(max(sp["m"], sp["p"])) + np.sqrt(sp["n"]))
            e = errors(got, ref, pinned(ref, sp["k"], nu))
            errs.append(dict(pair=i, m=sp["m"], p=sp["p"], n=sp["n"], k=sp["k"], **e))
            worst = max(worst, e["theta_pinned"])
        cpu = {"value": len(sample) / tcpu, "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{len(sample)} of the 256 pairs (every 32nd), {tcpu:.1f}s, NumPy/LAPACK FP64"}
        gate = bool(worst <= 1e-4)
        log(f"[bench] batch: oracle on {len(sample)} pairs: worst pinned theta error {worst:.2e}")
    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": "batch of 256 uneven pairs: m, p in [2000, 20000], n in [50, 500], shared rank "
                               "10..50, decays 0.6..0.95, noise 1e-5, FP32, BF16 sketches, oversample 10, q=2, "
                               "one captured graph",
                   "pairs": len(specs), "power_iters": q, "path": "mixed"},
        "autotune": tune,
        "accuracy_gate_passed": gate,
        "roofline": roof,
        "cpu_baseline": cpu,
        "errors_vs_oracle_sample": errs,
    }
    print(json.dumps(out), flush=True)


def time_path(R, torch, dev, G1, G2, m, p, n, k, o, q, seed, dt, prec, args):
    """Autotune, warm up and time one precision path on the device pair;
    returns its timings, per-stage profile and outputs (host arrays)."""
    plan = R.Plan(R.make_desc(m, p, n, k, o, q, seed, dt, prec), dev)
    outs = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev, uvr=True)
    tune = None
    if not args.no_tune:
        choice, tms = R.autotune(plan, G1, G2, outs, reps=2)
        tune = {"rows_per_tile": choice[0], "cols_per_lane": choice[1],
                "chunks": ["heuristic", "half", "twice"][choice[2]],
                "kernels": {0: None, 1: "8-wave k_nn/k_tn", 2: "per-wave k_gw/k_gtq"}[choice[3]], "ms": tms}
        log(f"[bench] {prec}: autotuned tile shapes {tune}")
    for _ in range(args.warmup):
        R.run(plan, G1, G2, outs)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        R.run(plan, G1, G2, outs)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # one profiled run: per-stage HIP events on the run's stream
    R.lib().rgsvd_profile(plan.h, 1)
    R.run(plan, G1, G2, outs)
    torch.cuda.synchronize()
    stages = R.profile_read(plan)
    R.lib().rgsvd_profile(plan.h, 0)
    got = {kk: v.cpu().numpy() for kk, v in outs.items()}
    agg = {}
    for tag, t in stages:
        a = agg.setdefault(tag, [0.0, 0])
        a[0] += t
        a[1] += 1
    sketch_ms = next(t for tag, t in stages if tag == "nn")
    log(f"[bench] {prec}: {ms:.3f} ms/pair ({1000 / ms:.1f} pairs/s); sketch {sketch_ms:.3f} ms;"
        f" info {got['info'].tolist()}")
    log("[bench]   stages: " + ", ".join(f"{kk}={v[0]:.3f}ms/{v[1]}" for kk, v in
                                        sorted(agg.items(), key=lambda x: -x[1][0])))
    del plan
    return dict(ms=ms, stages=agg, stage_list=stages, sketch_ms=sketch_ms, got=got,
                info=got["info"].tolist(), tune=tune)


def train_sizing_network(dev):
    """The sizing network trained as the library's gain test trains it: 176
    pairs of the training recipe (sizing.TRAIN_RANGES, seed 21) and 24 at
    the workload's scale (sizing.TRAIN_LARGE, seed 121), labelled on the GPU
    by the method itself, unpinned pairs left out, 600 full-batch Adam steps
    of the library's HIP kernels.  Returns (params, training pairs,
    seconds)."""
    import torch
    from paper_2404_09459_amd import sizing as S
    t0 = time.time()

    def small(s):
        G1, G2 = S.make_pair(s)
        return torch.from_numpy(G1).to(dev), torch.from_numpy(G2).to(dev)

    X, T, _ = S.label_set(dev, S.pair_specs(240, seed=21, **S.TRAIN_RANGES)[:176], small)
    X2, T2, _ = S.label_set(dev, S.pair_specs(24, seed=121, **S.TRAIN_LARGE), lambda s: S.make_pair_device(s, dev))
    X, T = X + X2, T + T2
    X = torch.tensor(np.array(X), dtype=torch.float32, device=dev)
    T = torch.tensor(np.array(T), dtype=torch.float32, device=dev)
    params, _ = S.train(X, T, dev, epochs=600, lr=3e-3, seed=2)
    torch.cuda.synchronize()
    return params, len(X), time.time() - t0


def time_learned(R, torch, dev, G1, G2, m, p, n, k, seed, dt, params, args):
    """Warm up and time the mixed-precision learned-sizing path."""
    plan = R.Plan(R.make_desc(m, p, n, k, 0, 0, seed, dt, "mixed", "learned"), dev)
    R.check(R.lib().rgsvd_set_sizing_model(plan.h, R._ptr(params), R._stream(dev)), "set model")
    outs = R.alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, dev, uvr=True)
    for _ in range(max(1, args.warmup)):
        R.run(plan, G1, G2, outs)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        R.run(plan, G1, G2, outs)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    got = {kk: v.cpu().numpy() for kk, v in outs.items()}
    log(f"[bench] mixed + learned: {ms:.3f} ms/pair ({1000 / ms:.1f} pairs/s); info {got['info'].tolist()}")
    del plan
    return dict(ms=ms, got=got, info=got["info"].tolist())


def time_batch_of_pairs(R, torch, dev, m, p, n, k, o, q, nu, dt, B, args):
    """B pairs of the workload's shape and spectrum (the recipe drawn on the
    device, seeds 31..31+B-1) in one batched plan, mixed precision, replayed
    as one graph: the rounds of the latency-bound small step of all B pairs
    share their launches.  Pair 0 is also run alone, and its angular
    distances compared with the batch's."""
    from paper_2404_09459_amd import inputs as I
    j = np.arange(k)
    pairs = [I.lowrank_pair_device(m, p, n, k, 0.97 ** j, 0.97 ** j, 31 + b, nu, dev) for b in range(B)]
    torch.cuda.synchronize()
    descs = [R.make_desc(m, p, n, k, o, q, 3, dt, "mixed") for _ in range(B)]
    plan = R.BatchPlan(descs, dev)
    outs = plan.bind(pairs)
    for _ in range(max(1, args.warmup)):
        plan.run()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, args.steps // 2)
    e0.record(st)
    for _ in range(steps):
        plan.run()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    got0 = outs[0]["theta"].cpu().numpy()
    info0 = outs[0]["info"].cpu().numpy().tolist()
    del plan, outs
    single = R.rgsvd(pairs[0][0], pairs[0][1], k, o, q, 3, precision="mixed")
    torch.cuda.synchronize()
    dth = float(np.max(np.abs(got0 - single["theta"].cpu().numpy())))
    del pairs, single
    torch.cuda.empty_cache()
    log(f"[bench] batch of {B} pairs: {ms:.3f} ms per batch ({1000 * B / ms:.1f} pairs/s); "
        f"pair 0 against its single run |dtheta| {dth:.1e}; info {info0}")
    return {"pairs": B, "ms_per_batch": ms, "pairs_per_s": 1000.0 * B / ms, "ms_per_pair": ms / B,
            "theta_vs_single_run": dth, "info_pair0": info0,
            "recipe": f"{B} pairs of the workload's recipe drawn on the device (torch generator, seeds 31..{30 + B})"}


def gate_of(e, k):
    """1e-4 on the pinned angular distances; 1e-5 on the entropies when every
    pair is pinned (D sums over all t pairs)."""
    return bool(e["theta_pinned"] <= 1e-4 and (e["D"] <= 1e-5 or e["n_pinned"] < k))


def roofline_of(dom_tag, dom_ms, dom_cnt, info, m, p, n, k, l, esz, flag, workload_name):
    """The dominant stage priced against the roofline that bounds it."""
    avg_ms = dom_ms / dom_cnt
    gbytes = (m + p) * n * esz
    N = 2 * l
    if dom_tag == "bjacobi":
        # block one-sided Jacobi on the factor of M (order N): a sweep visits
        # the N (N - 1) / 2 column pairs, each with three length-N inner
        # products and a rotation of two length-N columns, 12 N flops; sweeps
        # as reported in info[5]
        sw1 = int(info[5])
        flops = sw1 * 6.0 * N * N * (N - 1)
        roof = {"bound": "alu", "achieved": flops / (dom_ms * 1e-3) / 1e12, "peak": FP64_VEC_PEAK_TF,
                "unit": "TFLOP/s", "traffic": TRAFFIC.get(workload_name, {}).get("bjacobi")}
    elif dom_tag == "small":
        # k_small (its launches summed): pivoted Cholesky of M (N^3 / 3),
        # H = L1^T L1 (l t (t + 1)), pivoted Cholesky of H (t^3 / 3), the
        # one-sided Jacobi on H's factor (info[6] sweeps of t (t - 1) / 2
        # pairs at 12 t flops), L Y (2 N t^2)
        t = k
        sw2 = int(info[6])
        flops = N ** 3 / 3.0 + l * t * (t + 1.0) + t ** 3 / 3.0 + sw2 * 6.0 * t * t * (t - 1) + 2.0 * N * t * t
        roof = {"bound": "alu", "achieved": flops / (dom_ms * 1e-3) / 1e12, "peak": FP64_VEC_PEAK_TF,
                "unit": "TFLOP/s", "traffic": TRAFFIC.get(workload_name, {}).get("small")}
    elif dom_tag == "chol":
        # Cholesky and inverse of the l x l Gram of both sides per launch:
        # l^3 / 3 + l^3 / 3 flops each
        flops = 2 * (2.0 * l ** 3 / 3.0)
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": FP64_VEC_PEAK_TF,
                "unit": "TFLOP/s", "traffic": None}
    elif dom_tag in ("nn", "tn") and flag == "mixed":
        roof = {"bound": "hbm", "achieved": gbytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "traffic": None}
    elif dom_tag in ("nn", "tn"):
        roof = {"bound": "mfma", "achieved": 2.0 * (m + p) * n * l / (avg_ms * 1e-3) / 1e12,
                "peak": MFMA_PEAK_TF[flag], "unit": "TFLOP/s", "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"] if roof.get("achieved") is not None else None
    roof["kernel"] = {"small": "k_small", "nn": "k_nn" if flag == "mixed" else "k_gw",
                      "tn": "k_tn" if flag == "mixed" else "k_gtq", "chol": "k_chol",
                      "bjacobi": "k_bjinit + k_bjround + k_bjsweep"}.get(dom_tag, dom_tag)
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = dom_cnt
    return roof


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "medium", "small", "batch256"],
                    help="large (default): the 100000/80000 x 2000 pair; medium: the 20000/15000 x 5000 "
                         "pair; batch256: 256 uneven pairs in one captured graph (its own JSON line)")
    ap.add_argument("--precisions", default="mixed,fp32,fp64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg and the accuracy gate")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-single-thread", action="store_true", help="skip the one-thread oracle timing")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile-shape autotuner")
    ap.add_argument("--batch-pairs", type=int, default=4,
                    help="large workload: also time a batched plan of this many pairs of the same shape "
                         "(0: skip)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the mixed + learned-sizing leg (it trains the sizing network first)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain elementwise copy of MIB MiB (read + write) for "
                         "calibrating hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build measures one MI355X "
              f"(the path runs on a single GPU; multi-GPU row sharding is not built)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        bench_batch(args)
        return

    import torch
    from paper_2404_09459_amd import rgsvd as R

    dev = torch.device("cuda:0")
    R.lib()
    t0 = time.time()
    w, nu = workload(args.workload)
    G1h, G2h = w["G1"], w["G2"]
    m, n = G1h.shape
    p = G2h.shape[0]
    k, o, q, seed = w["k"], w["oversample"], w["q"], w["seed"]
    l = k + o
    esz = G1h.dtype.itemsize
    dt = R.F64 if esz == 8 else R.F32
    log(f"[bench] workload {w['name']} generated in {time.time() - t0:.1f}s")
    G1 = torch.from_numpy(G1h).to(dev)
    G2 = torch.from_numpy(G2h).to(dev)
    torch.cuda.synchronize()

    precs = [x for x in args.precisions.split(",") if x]
    res = {prec: time_path(R, torch, dev, G1, G2, m, p, n, k, o, q, seed, dt, prec, args) for prec in precs}
    learned, net, net_params = None, None, None
    if not args.no_learned and esz == 4:
        params, ntrain, tsec = train_sizing_network(dev)
        net_params = params
        net = {"training_pairs": ntrain, "training_seconds": round(tsec, 1),
               "recipe": "176 pairs m, p in [1000, 4000], n in [200, 1000], rank 5..220 and 24 pairs m, p in "
                         "[20000, 100000], n in [1000, 2000], rank 50..220; last-component magnitude 1e-4..0.3, "
                         "noise floor nu 1e-6..1e-2, k = components above 2 nu; labelled on the GPU by the "
                         "method, unpinned left out; 600 Adam steps of the HIP MLP kernels"}
        log(f"[bench] sizing network trained on {ntrain} pairs in {tsec:.1f}s")
        learned = time_learned(R, torch, dev, G1, G2, m, p, n, k, seed, dt, params, args)

    batch = None
    if args.workload == "large" and args.batch_pairs > 0 and esz == 4 and "mixed" in res:
        batch = time_batch_of_pairs(R, torch, dev, m, p, n, k, o, q, nu, dt, args.batch_pairs, args)

    if args.calib_copy > 0:
        nel = args.calib_copy * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: 3 x {args.calib_copy} MiB read + {args.calib_copy} MiB written")
        del a, b

    # ---------------------------------------------------------- CPU oracle --
    flag = "mixed" if "mixed" in res else precs[0]
    cpu, ref, distinct = None, None, None
    if not args.no_cpu:
        G1d = G1h.astype(np.float64)
        G2d = G2h.astype(np.float64)
        tall, ref = time_oracle(G1d, G2d, k, o, q, seed, args.cpu_reps)
        cpu = {"value": 1.0 / tall, "unit": "pairs/s", "cores": int(oracle_threads()), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{max(1, args.cpu_reps)} full pairs of the workload (median {tall:.2f}s each), "
                         f"NumPy/LAPACK FP64 on the host, all BLAS threads"}
        if not args.no_single_thread:
            t1, _ = time_oracle(G1d, G2d, k, o, q, seed, 1, threads=1)
            cpu["single_thread"] = {"value": 1.0 / t1, "unit": "pairs/s", "cores": 1,
                                    "sample": f"1 full pair ({t1:.2f}s), BLAS/LAPACK limited to one thread"}
        if learned is not None:
            # parity of the learned run: the oracle at the (l, q) it chose
            ll, lq = int(learned["info"][1]), int(learned["info"][3])
            refl = O_rgsvd(G1d, G2d, k, ll - k, lq, seed)
            el = errors(learned["got"], refl, pinned(refl, k, nu))
            learned["parity"] = {"reference": f"oracle FP64 at the chosen l={ll}, q={lq}", "errors": el,
                                 "gate_passed": gate_of(el, k)}
            log(f"[bench] learned vs oracle at its sizes: {el}")
        del G1d, G2d
        # the same shapes with distinct decays: the mixed path against the
        # full-size oracle on spread-out GSVs
        wd, _ = workload(args.workload, distinct=True)
        g1d = torch.from_numpy(wd["G1"]).to(dev)
        g2d = torch.from_numpy(wd["G2"]).to(dev)
        rd = time_path(R, torch, dev, g1d, g2d, m, p, n, k, o, q, seed, dt, flag, args)
        ldist = time_learned(R, torch, dev, g1d, g2d, m, p, n, k, seed, dt, net_params, args) \
            if learned is not None else None
        del g1d, g2d
        refd = O_rgsvd(wd["G1"].astype(np.float64), wd["G2"].astype(np.float64), k, o, q, seed)
        ed = errors(rd["got"], refd, pinned(refd, k, nu))
        if ldist is not None:
            # whether the learned sizes are enough: on the pair with spread-out
            # GSVs, against a converged run of the method (the oracle at
            # l = min(2k + 50, 224), q = 4), the default sizes beside it
            lc = min(2 * k + 50, m, p, n, 224)
            refc = O_rgsvd(wd["G1"].astype(np.float64), wd["G2"].astype(np.float64), k, lc - k, 4, seed)
            idc = pinned(refc, k, nu)
            e_l = errors(ldist["got"], refc, idc)
            e_d = errors(rd["got"], refc, idc)
            learned["sizing"] = {"workload": "the distinct-decay pair", "reference": f"oracle FP64, l={lc}, q=4",
                                 "l_q_chosen": [int(ldist["info"][1]), int(ldist["info"][3])],
                                 "ms_per_pair": ldist["ms"], "errors_learned": e_l,
                                 "errors_default_sizes": e_d, "gate_passed": gate_of(e_l, k)}
            log(f"[bench] distinct pair, learned {ldist['info'][1]}/{ldist['info'][3]} vs converged: {e_l}; "
                f"default sizes vs converged: {e_d}")
        distinct = {"workload": wd["name"] + f" (G2 decay {0.96 if args.workload == 'large' else 0.93})",
                    "path": flag, "ms_per_pair": rd["ms"], "errors_vs_oracle": ed,
                    "theta_range": [float(np.min(refd["theta"])), float(np.max(refd["theta"]))],
                    "gate_passed": gate_of(ed, k)}
        log(f"[bench] distinct-decay gate: {ed}")

    # ------------------------------------------------------------ report --
    ms = res[flag]["ms"]
    sk_flops = 2.0 * (m + p) * n * l
    paths = {}
    for prec, r in res.items():
        e = errors(r["got"], ref, pinned(ref, k, nu)) if ref is not None else None
        paths[prec] = {"pairs_per_s": 1000.0 / r["ms"], "ms_per_pair": r["ms"],
                       "sketch_tflops": sk_flops / (r["sketch_ms"] * 1e-3) / 1e12,
                       "errors_vs_oracle": e, "gate_passed": gate_of(e, k) if e else None,
                       "info": r["info"], "autotune": r["tune"],
                       "stage_ms": {kk: round(v[0], 4) for kk, v in r["stages"].items()}}
    if learned is not None:
        par, siz = learned.get("parity"), learned.get("sizing")
        paths["mixed_learned"] = {"pairs_per_s": 1000.0 / learned["ms"], "ms_per_pair": learned["ms"],
                                  "parity": par, "sizing": siz,
                                  "gate_passed": bool(par["gate_passed"] and siz["gate_passed"]) if par and siz
                                  else None,
                                  "info": learned["info"], "l_q_chosen": [learned["info"][1], learned["info"][3]],
                                  "sizing_network": net}
    # dominant kernel of the headline path: each stage's event time carries
    # the cost of an empty launch between events (the smallest stage time),
    # so stages are ranked by their time above it
    agg = res[flag]["stages"]
    floor = min(t for _, t in res[flag]["stage_list"])
    dom_tag, (dom_ms, dom_cnt) = max(agg.items(), key=lambda x: x[1][0] - x[1][1] * floor)
    roof = roofline_of(dom_tag, dom_ms, dom_cnt, res[flag]["info"], m, p, n, k, l, esz, flag, args.workload)
    # the streaming sketch kernel beside it: one read of G1 and G2 per launch
    gbytes = (m + p) * n * esz
    sk_ms = res[flag]["sketch_ms"]
    roof_sketch = {"bound": "hbm", "kernel": "k_nn" if flag == "mixed" else "k_gw",
                   "achieved": gbytes / (sk_ms * 1e-3) / 1e9,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbytes / (sk_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "traffic": TRAFFIC.get(args.workload, {}).get("sketch") if flag == "mixed" else None,
                   "tflops": sk_flops / (sk_ms * 1e-3) / 1e12,
                   "bf16_mfma_frac": sk_flops / (sk_ms * 1e-3) / 1e12 / MFMA_PEAK_TF["mixed"]}
    gate = None
    if paths[flag]["gate_passed"] is not None:
        gate = bool(paths[flag]["gate_passed"] and (distinct is None or distinct["gate_passed"]))
    out = {
        "metric": METRIC, "value": 1000.0 / ms, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32+f64" if flag == "mixed" else {"fp32": "f32", "fp64": "f64"}[flag],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: G1 {m}x{n}, G2 {p}x{n}, k={k}, oversample={o}, q={q}",
                   "m": m, "p": p, "n": n, "k": k, "oversample": o, "power_iters": q,
                   "storage": str(G1h.dtype), "path": flag},
        "accuracy_gate_passed": gate,
        "sketch_tflops": paths[flag]["sketch_tflops"],
        "mixed_vs_fp64_speedup": (res["fp64"]["ms"] / res["mixed"]["ms"]) if {"mixed", "fp64"} <= set(res) else None,
        "mixed_learned_vs_fp64_speedup": (res["fp64"]["ms"] / learned["ms"])
        if (learned is not None and "fp64" in res) else None,
        "roofline": roof,
        "roofline_sketch": roof_sketch,
        "cpu_baseline": cpu,
        "paths": paths,
        "batch_of_pairs": batch,
        "distinct_decay_gate": distinct,
    }
    print(json.dumps(out), flush=True)


def O_rgsvd(*a, **kw):
    from oracle import rgsvd as O
    return O.rgsvd(*a, **kw)


if __name__ == "__main__":
    main()
