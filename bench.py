"""Benchmark: A + A* operator pairs per second at 256^2 FP32, batched vs single.

Workload (default): the limited-view geometry -- 256 x 256 image on [-1,1]^2
(zero outside r < 0.9), 256 detectors on a 180 degree arc of the unit circle,
512 time samples on (0, 2], c = 1 -- with a batch of 64 seeded phantoms
(20 Gaussian blobs, 3 discs, 4 thin line segments each) and noisy data
(1 % of max|g|).  One step = one pat_forward over the batch plus one
pat_adjoint over the batch; `value` counts operator pairs (instances) per
second.  The single-instance rate (batch 1, same geometry) is reported beside
it.  Before timing, instance 0 is checked against the FP64 oracle (relative
L2 <= 1e-5); that oracle run, timed on the host cores, is the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "A+A* operator pairs/sec at 256² FP32 (rel L2 ≤1e-5 vs FP64); batched vs single"
HBM_PEAK_GBS = 8000.0
FWD_NAMES = ["colpass_fwd", "rowpass_fwd", "gather", "ring_fwd", "dct_fwd"]
ADJ_NAMES = ["dct_adj", "ring_adj", "spread", "rowpass_adj", "colpass_adj"]


def algorithmic_bytes(info, geom):
    """Compulsory HBM bytes per instance of each kernel: every input element
    read once, every output element written once (tables not counted)."""
    N, D, T = geom.n, geom.n_det, geom.n_t
    Ng = info.n_grid
    Hy = Ng // 2 + 9
    P = info.n_points
    NL = info.n_lam
    c8 = 8
    return {
        "colpass_fwd": 4 * N * N + c8 * Hy * N,
        "rowpass_fwd": c8 * Hy * N + c8 * Hy * Ng,
        "gather": c8 * Hy * Ng + 24 * P + c8 * P,
        "ring_fwd": c8 * P + 4 * D * NL,
        "dct_fwd": 4 * D * NL + 4 * D * T,
        "dct_adj": 4 * D * T + 4 * D * NL,
        "ring_adj": 4 * D * NL + 12 * P + c8 * P,
        "spread": c8 * P + 16 * P + c8 * Hy * Ng,
        "rowpass_adj": c8 * Hy * Ng + c8 * Hy * N,
        "colpass_adj": c8 * Hy * N + 4 * N * N,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the operator pair shards by instance with no "
              "communication, so --gpus %d is not run (see DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import CONFIGS, add_noise, config_geometry, make_phantom

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    cfg = CONFIGS[2]
    geom = config_geometry(2)
    B = args.batch
    nb, nd, nl = cfg["phantom"]
    print("bench: building inputs (batch %d)" % B, file=sys.stderr, flush=True)
    fs = np.stack([make_phantom(geom.n, nb, nd, nl, cfg["seed"] + 1000 * b) for b in range(B)])
    plan = pat.PatPlan(geom, max_batch=B)
    plan1 = pat.PatPlan(geom, max_batch=1)
    f = torch.tensor(fs, dtype=torch.float32, device=dev)
    g_clean = plan.forward(f)
    torch.cuda.synchronize()
    gm = np.stack([add_noise(g_clean[b].cpu().double().numpy(), cfg["noise"], cfg["seed"] + 1000 * b)
                   for b in range(B)])
    g_meas = torch.tensor(gm, dtype=torch.float32, device=dev)
    g_out = torch.empty_like(g_meas)
    f_out = torch.empty_like(f)

    # ---- parity of instance 0 against the FP64 oracle (also the CPU baseline) ----
    parity = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        print("bench: oracle parity + CPU baseline", file=sys.stderr, flush=True)
        nthreads = oracle.get_threads()
        reps, t_cpu = 0, 0.0
        while True:
            t0 = time.perf_counter()
            ref_g = oracle.forward(geom, fs[0])
            ref_f = oracle.adjoint(geom, gm[0])
            t_cpu += time.perf_counter() - t0
            reps += 1
            if t_cpu >= 10.0 or reps >= 3:
                break
        g0 = plan.forward(f[0:1].contiguous())[0].cpu().double().numpy()
        a0 = plan.adjoint(g_meas[0:1].contiguous())[0].cpu().double().numpy()
        parity = {
            "fwd_rel_l2": float(np.linalg.norm(g0 - ref_g) / np.linalg.norm(ref_g)),
            "adj_rel_l2": float(np.linalg.norm(a0 - ref_f) / np.linalg.norm(ref_f)),
        }
        assert parity["fwd_rel_l2"] <= 1e-5 and parity["adj_rel_l2"] <= 1e-5, parity
        cpu = {"value": reps / t_cpu, "unit": "pairs/s", "cores": nthreads, "kind": "oracle",
               "sample": "%d x (one A + one A*) on instance 0 of the 256^2 workload, FP64 direct sums" % reps}

    stream = torch.cuda.current_stream(dev)

    def step(p, fin, gin, gout, fout):
        p.forward(fin, out=gout)
        p.adjoint(gin, out=fout)

    # ---- batched ----
    print("bench: timing batched", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(plan, f, g_meas, g_out, f_out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step(plan, f, g_meas, g_out, f_out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = B * 1000.0 / ms_step

    # ---- single instance ----
    print("bench: timing single", file=sys.stderr, flush=True)
    f1, g1 = f[0:1].contiguous(), g_meas[0:1].contiguous()
    go1, fo1 = torch.empty_like(g1), torch.empty_like(f1)
    for _ in range(args.warmup):
        step(plan1, f1, g1, go1, fo1)
    torch.cuda.synchronize()
    s_steps = max(args.steps, 20)
    e0.record(stream)
    for _ in range(s_steps):
        step(plan1, f1, g1, go1, fo1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / s_steps

    # ---- per-kernel durations (HIP events around each launch, same launches) ----
    pat.pat_profile_enable(plan.handle, True)
    nprof = 10
    acc_f = [0.0] * len(FWD_NAMES)
    acc_a = [0.0] * len(ADJ_NAMES)
    for _ in range(nprof):
        plan.forward(f, out=g_out)
        ms = pat.pat_profile_read(plan.handle, 0)
        acc_f = [a + b for a, b in zip(acc_f, ms)]
        plan.adjoint(g_meas, out=f_out)
        ms = pat.pat_profile_read(plan.handle, 1)
        acc_a = [a + b for a, b in zip(acc_a, ms)]
    pat.pat_profile_enable(plan.handle, False)
    kms = {n: v / nprof for n, v in zip(FWD_NAMES + ADJ_NAMES, acc_f + acc_a)}
    abytes = algorithmic_bytes(plan.info, geom)
    dom = max(kms, key=kms.get)
    achieved = abytes[dom] * B / (kms[dom] * 1e-3) / 1e9
    gbs = {n: abytes[n] * B / (kms[n] * 1e-3) / 1e9 for n in kms}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "limited-view 256x256, 256 detectors on a 180 deg arc, 512 samples on (0,2], "
                               "batch %d; step = A then A* over the batch" % B,
                   "n": geom.n, "n_det": geom.n_det, "n_t": geom.n_t, "arc_deg": 180, "batch": B},
        "single": {"value": round(1000.0 / ms_single, 1), "unit": "pairs/s", "ms_per_pair": round(ms_single, 4),
                   "batch": 1},
        "batched_over_single": round(value * ms_single / 1000.0, 2),
        "wall_s_timed": round(wall, 3),
        "parity": parity,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "kernels_ms": {k: round(v, 4) for k, v in kms.items()},
        "kernels_gbs": {k: round(v, 1) for k, v in gbs.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    plan1.close()


if __name__ == "__main__":
    main()
