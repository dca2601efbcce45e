"""Benchmark: A + A* operator pairs per second at 256^2 FP32, batched vs single.

Default workload: the limited-view geometry -- 256 x 256 image on [-1,1]^2
(zero outside r < 0.9), 256 detectors on a 180 degree arc of the unit circle,
512 time samples on (0, 2], c = 1 -- with a batch of 64 seeded phantoms
(20 Gaussian blobs, 3 discs, 4 thin line segments each) and noisy data
(1 % of max|g|).  One step = one pat_forward over the batch plus one
pat_adjoint over the batch; `value` counts operator pairs (instances) per
second.  The single-instance rate (batch 1, same geometry) is reported beside
it.  Before timing, instance 0 is checked against the FP64 oracle (relative
L2 <= 1e-5); that oracle run, timed on the host cores, is the CPU baseline.

Other workloads (one JSON line each; not the default):
  --workload mixed   64 heterogeneous instances (N 128..512, D 64..512, arcs 90..360 deg)
                     batched vs per-instance launches, eager and graph-captured
  --workload tv3     TV projected-gradient iterations/s at 256^2, 128 detectors on 120 deg
  --workload large   1024^2, 1024 detectors on 270 deg, 2048 samples, batch 8:
                     TV iterations/s and staged HBM GB/s
  --workload paper   the paper's timed shape (760^2, 256 detectors on 270 deg, 2030 samples)
  --workload pdhg3   primal-dual TV (the paper's TV baseline) at 256^2, 128 detectors on 120 deg,
                     run to relative change <= 1e-4: iterations/s and time to solution
  --workload pdhg-large  the same at 1024^2, 1024 detectors on 270 deg, batch 8
      (with --sim-data, both primal-dual workloads reconstruct from data the FFT
      wave-propagation simulator computed on a grid twice as fine)
  --workload cgls    CGLS steps/s on the default workload (two steps per HIP graph)
  --workload dip     deep-image-prior iterations/s at the paper's timed shape
  --workload dense   the default workload with jittered explicit detector angles
                     (dense angular synthesis on the matrix cores)
  --workload sim     FFT wave-propagation data simulations/s on the 512^2 fine grid

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--workload ...] [--sim-data]
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
FP32_PEAK_TFLOPS = 157.3           # published FP32 vector peak (packed FP32)
FP32_NONPACKED_TFLOPS = 78.6       # ceiling of code built without packed FP32
FWD_NAMES = ["colpass_fwd", "rowpass_fwd", "gather", "ring_fwd", "dct_fwd"]
ADJ_NAMES = ["dct_adj", "ring_adj", "spread", "rowpass_adj", "colpass_adj"]
# kernel symbols (without template arguments) of each timed stage; the
# compile-time-length variants where a plan has them
KERNEL_SYMBOL = {"colpass_fwd": ("k_colpass_fwd",), "rowpass_fwd": ("k_rowpass_fwd",), "gather": ("k_gather",),
                 "ring_fwd": ("k_ring_fwd", "k_ring_fwd_spec"), "dct_fwd": ("k_dct_det", "k_dct_spec"),
                 "dct_adj": ("k_dct_det", "k_dct_spec"), "ring_adj": ("k_ring_adj", "k_ring_adj_spec"),
                 "spread": ("k_spread",), "rowpass_adj": ("k_rowpass_adj",), "colpass_adj": ("k_colpass_adj",),
                 "syn_fwd": ("k_syn_dense_fwd",), "syn_adj": ("k_syn_dense_adj",)}
MFMA_FP32_PEAK_TFLOPS = 157.3   # dense FP32 matrix-core peak of the MI355X
# interpolation or spread of one polar point: 16 kernel evaluations (~6 flops),
# 64 weight products and 64 complex x real multiply-adds (4 flops)
FLOPS_PER_POINT = 16 * 6 + 64 + 64 * 4
CALIB_ELEMS = 256 * 1024 * 1024    # float32 elements of the calibration copies (1 GiB each way)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2604_19176_amd", "csrc", "kernels.hip")


def kernels_hash():
    """Hash of the device sources (kernels.hip and the headers it includes)."""
    from paper_2604_19176_amd.profiling import source_hash
    return source_hash(KERNEL_SRC)


def algorithmic_bytes(info, geom, B):
    """Compulsory HBM bytes of one launch of each kernel over B instances of
    one plan: every instance's own inputs read once and outputs written once
    (B times), plus each plan table the kernel reads counted once per launch
    (the instances share it).  Workspace the staging alone adds (the spread's
    partial rows, tile halos) is not counted."""
    N, D, T = geom.n, geom.n_det, geom.n_t
    Ng = info.n_grid
    Hy = Ng // 2 + 9
    NB = Ng // 2 + 2
    P = info.n_points
    NL = info.n_lam
    KM = info.n_ring_modes                 # sum over rings of the modes kept
    c8 = 8
    inst = {
        "colpass_fwd": 4 * N * N + c8 * Hy * N + 4 * N,     # f; column spectra; per-column mass sums
        "rowpass_fwd": c8 * Hy * N + c8 * Hy * Ng,
        "gather": c8 * Hy * Ng + c8 * P,                    # spectrum; polar values
        "ring_fwd": c8 * P + 4 * D * NL,                    # polar values; ring output at the detectors
        "dct_fwd": 4 * D * NL + 4 * D * T + 4 * N,
        "dct_adj": 4 * D * T + 4 * D * NL + 4 * D,
        "ring_adj": 4 * D * NL + c8 * P,
        "spread": c8 * P + c8 * Hy * Ng,
        "rowpass_adj": c8 * Hy * Ng + c8 * Hy * N,
        "colpass_adj": c8 * Hy * N + 4 * N * N + 4 * D,
    }
    image_tab = 4 * N + 8 * N                               # deapodisation, mask row ranges
    band_tab = 4 * NB * (Ng + 1)                            # band CSR
    ring_tab = c8 * KM + 16 * NL                            # mode coefficients; ring offsets, K_n, descriptors
    table = {
        "colpass_fwd": image_tab, "rowpass_fwd": 0,
        "gather": 16 * P + c8 * P + band_tab,               # band-order geometry and half-pixel phase
        "ring_fwd": ring_tab,
        "dct_fwd": 0, "dct_adj": 0,
        "ring_adj": ring_tab + 4 * P,                       # band-order slot per point
        "spread": 16 * P + c8 * P + band_tab,               # band-order geometry and half-pixel phase
        "rowpass_adj": 0, "colpass_adj": image_tab,
    }
    return {k: B * inst[k] + table[k] for k in inst}


def algorithmic_flops(info, geom, name):
    """Nominal FP32 flops per instance of the compute-bound kernels."""
    P, NL, D = info.n_points, info.n_lam, geom.n_det
    if name in ("gather", "spread"):
        return FLOPS_PER_POINT * P
    if name in ("ring_fwd", "ring_adj"):
        ring = P / max(NL, 1)                  # average half-ring length
        syn = 0 if info.syn_dense else max(info.len_czt, 2)
        return 5.0 * P * math.log2(max(ring, 2)) + (5.0 * NL * syn * math.log2(syn) / 2 if syn else 0.0)
    if name in ("syn_fwd", "syn_adj"):
        # dense synthesis: 2 (K_n + 1) real coefficients x D detectors per ring, one multiply-add each
        return 4.0 * info.n_ring_modes * D
    return None


def measured_traffic(dom, B):
    """HBM bytes per launch of kernel `dom` from the committed counter summary,
    or None when it was taken at another batch or from other device sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernels_hash") != kernels_hash() or tr.get("batch") != B:
            return None
        for name, d in tr.get("kernels", {}).items():
            if name.split("<")[0] in KERNEL_SYMBOL[dom]:
                return int(d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"])
    except (OSError, ValueError, KeyError, AttributeError):
        pass
    return None


def roofline(kms, info, geom, B, copy_gbs=None):
    """Roofline entry for the kernel with the largest per-launch time.  A
    kernel with nominal flops is ALU-bound when its flops per algorithmic byte
    exceed the ridge point of the FP32 rate this build can issue (packed FP32
    is off, so 78.6 TFLOP/s) over HBM's 8 TB/s; otherwise it is HBM-bound."""
    dom = max(kms, key=kms.get)
    t = kms[dom] * 1e-3
    traffic = measured_traffic(dom, B)
    fl = algorithmic_flops(info, geom, dom)
    ridge = FP32_NONPACKED_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if fl is not None and dom.startswith("syn_"):
        flops = fl * B
        ach = flops / t / 1e12
        return {"bound": "mfma", "kernel": dom, "achieved": round(ach, 3), "peak": MFMA_FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / MFMA_FP32_PEAK_TFLOPS, 4), "flops_per_launch": int(flops),
                "avg_launch_ms": round(kms[dom], 4), "traffic": traffic}
    byt = algorithmic_bytes(info, geom, B)[dom]
    if fl is not None and fl * B / byt > ridge:
        flops = fl * B
        ach = flops / t / 1e12
        return {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                "frac_of_nonpacked_78.6": round(ach / FP32_NONPACKED_TFLOPS, 4),
                "flops_per_launch": int(flops), "avg_launch_ms": round(kms[dom], 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": byt}
    ach = byt / t / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": byt, "avg_launch_ms": round(kms[dom], 4),
           "traffic": traffic}
    if copy_gbs:
        out["frac_of_measured_copy"] = round(ach / copy_gbs, 4)
    if fl is not None:  # below the ridge point: the nominal flops for reference
        out["flops_per_launch"] = int(fl * B)
        out["flops_per_byte"] = round(fl * B / byt, 2)
    return out


def kernel_times(pat, plan, f, g, gout, fout, nprof=10):
    """Average per-launch milliseconds of each kernel, from the library's HIP
    events recorded on the stream the kernels run on."""
    fwd, adj = FWD_NAMES, ADJ_NAMES
    if plan.info.syn_dense:  # explicit detector angles: the dense synthesis has its own slot
        fwd = FWD_NAMES[:4] + ["syn_fwd"] + FWD_NAMES[4:]
        adj = ADJ_NAMES[:1] + ["syn_adj"] + ADJ_NAMES[1:]
    pat.pat_profile_enable(plan.handle, True)
    acc_f = [0.0] * len(fwd)
    acc_a = [0.0] * len(adj)
    for _ in range(nprof):
        plan.forward(f, out=gout)
        acc_f = [a + b for a, b in zip(acc_f, pat.pat_profile_read(plan.handle, 0))]
        plan.adjoint(g, out=fout)
        acc_a = [a + b for a, b in zip(acc_a, pat.pat_profile_read(plan.handle, 1))]
    pat.pat_profile_enable(plan.handle, False)
    return {n: v / nprof for n, v in zip(fwd + adj, acc_f + acc_a)}


def time_pairs(torch, plan, f, g, gout, fout, steps, warmup):
    stream = torch.cuda.current_stream(plan.device)
    for _ in range(warmup):
        plan.forward(f, out=gout)
        plan.adjoint(g, out=fout)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.forward(f, out=gout)
        plan.adjoint(g, out=fout)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t0


def time_graph(torch, dev, fn, steps, warmup=2, per_graph=1):
    """Milliseconds per call of fn(), captured per_graph times into one
    CUDA/HIP graph that is replayed `steps` times."""
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream(dev).wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            fn()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    del graph
    return e0.elapsed_time(e1) / (steps * per_graph)


def time_eager(torch, dev, fn, steps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def copy_calibration(torch, dev):
    """The library's streaming copy over CALIB_ELEMS float32 (1 GiB read,
    1 GiB written, the size measure_copy times) and its 8-byte scatter over
    the same bytes: copies of known size whose byte counters calibrate the PMC
    traffic figures."""
    import paper_2604_19176_amd as pat
    x = torch.ones(CALIB_ELEMS, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    st = pat._stream(dev)
    pat.pat_stream_copy(x.data_ptr(), y.data_ptr(), 4 * CALIB_ELEMS, None, st)
    perm = torch.randperm(CALIB_ELEMS // 2, device=dev, dtype=torch.int64).to(torch.int32)
    pat.pat_stream_copy(x.data_ptr(), y.data_ptr(), 4 * CALIB_ELEMS, perm.data_ptr(), st)
    torch.cuda.synchronize()
    del x, y, perm


def measure_copy(torch, dev, nbytes=1 << 30, reps=20):
    """GB/s (read + write bytes / time) of the library's streaming copy over
    `nbytes` (1 GiB each way), best of `reps` launches timed with HIP events
    on the launch stream."""
    import paper_2604_19176_amd as pat
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    st = pat._stream(dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(3):
        pat.pat_stream_copy(x.data_ptr(), y.data_ptr(), nbytes, None, st)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pat.pat_stream_copy(x.data_ptr(), y.data_ptr(), nbytes, None, st)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    ok = bool(torch.equal(x[:1 << 20], y[:1 << 20])) and bool(torch.equal(x[-(1 << 20):], y[-(1 << 20):]))
    del x, y
    return {"gbs": round(2.0 * nbytes / (best * 1e-3) / 1e9, 1), "bytes_each_way": nbytes, "best_ms": round(best, 4),
            "kernel": "k_stream_copy", "copied_correctly": ok}


def step_roofline(kms, info, geom, B, ms_step, copy_gbs=None):
    """The whole A + A* step: the sum of every kernel's algorithmic bytes per
    launch (algorithmic_bytes) over the measured step time."""
    ab = algorithmic_bytes(info, geom, B)
    byt = sum(ab[k] for k in kms if k in ab)
    ach = byt / (ms_step * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_step": int(byt), "ms_per_step": round(ms_step, 4)}
    if copy_gbs:
        out["frac_of_measured_copy"] = round(ach / copy_gbs, 4)
    return out


def make_inputs(np, torch, plan, geom, cfg, B, dev, seed_stride):
    from pat_inputs import add_noise, make_phantom
    nb, nd, nl = cfg["phantom"]
    seeds = [cfg["seed"] + seed_stride * b for b in range(B)]
    fs = np.stack([make_phantom(geom.n, nb, nd, nl, s) for s in seeds])
    f = torch.tensor(fs, dtype=torch.float32, device=dev)
    g_clean = plan.forward(f)
    torch.cuda.synchronize()
    gm = np.stack([add_noise(g_clean[b].cpu().double().numpy(), cfg["noise"], s) for b, s in enumerate(seeds)])
    return fs, f, gm, torch.tensor(gm, dtype=torch.float32, device=dev)


def make_sim_inputs(np, torch, geom, cfg, B, dev, seed_stride):
    """Like make_inputs, but the clean data come from the wave-propagation
    simulator on a grid twice as fine (the same phantoms rendered at 2N), so
    they are free of the operator's own discretisation (no inverse crime)."""
    import paper_2604_19176_amd as pat
    from pat_inputs import add_noise, make_phantom
    nb, nd, nl = cfg["phantom"]
    seeds = [cfg["seed"] + seed_stride * b for b in range(B)]
    fs = np.stack([make_phantom(geom.n, nb, nd, nl, s) for s in seeds])
    sim = pat.PatSim(geom.with_(n=2 * geom.n))
    g_clean = [sim.run(torch.tensor(make_phantom(2 * geom.n, nb, nd, nl, s), dtype=torch.float32, device=dev))
               for s in seeds]
    torch.cuda.synchronize()
    sim.close()
    gm = np.stack([add_noise(g_clean[b].cpu().double().numpy(), cfg["noise"], s) for b, s in enumerate(seeds)])
    return fs, torch.tensor(fs, dtype=torch.float32, device=dev), gm, torch.tensor(gm, dtype=torch.float32, device=dev)


GOLDEN_LARGE = os.path.join(ROOT, "tests", "golden", "large_1024.npz")


def parity_against_oracle(np, geom, fs, gm, g_out, f_out, idx):
    """Relative L2 of the timed batch outputs (A f and A* g_meas, instances
    `idx`) against the FP64 oracle, and the oracle's wall time for them."""
    import oracle
    errs, t_cpu = [], 0.0
    for b in idx:
        t0 = time.perf_counter()
        ref_g = oracle.forward(geom, fs[b])
        ref_f = oracle.adjoint(geom, gm[b])
        t_cpu += time.perf_counter() - t0
        gb = g_out[b].cpu().double().numpy()
        ab = f_out[b].cpu().double().numpy()
        errs.append({"instance": int(b),
                     "fwd_rel_l2": float(np.linalg.norm(gb - ref_g) / np.linalg.norm(ref_g)),
                     "adj_rel_l2": float(np.linalg.norm(ab - ref_f) / np.linalg.norm(ref_f))})
    return errs, t_cpu, oracle.get_threads()


def large_leg(args, np, torch, pat, dev):
    """The 1024^2 workload (1024 detectors on a 270 deg arc, 2048 samples,
    batch 8, 1 % noise): the projected-gradient TV loop (A, residual, A*, TV
    gradient, update per iteration, HIP graphs of 10 iterations) over
    `--large-steps` iterations, its per-kernel times and roofline, and
    instance 0 of the timed launch shapes against the stored FP64 oracle values
    (every 16th detector's trace of A f, A* d at 4000 pixels)."""
    from paper_2604_19176_amd.recon import TVReconstructor
    from pat_inputs import CONFIGS, config_geometry
    cfg = CONFIGS[5]
    geom = config_geometry(5)
    B = cfg["batch"]
    print("bench: large workload (1024^2, batch %d)" % B, file=sys.stderr, flush=True)
    plan = pat.PatPlan(geom, max_batch=B)
    fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, 1)
    launch = plan.autotune(batch=B, cache_path=args.tune_cache) if args.tune else plan.launch
    g_out, f_out = torch.empty_like(g_meas), torch.empty_like(f)
    parity = None
    if os.path.exists(GOLDEN_LARGE):
        gold = np.load(GOLDEN_LARGE)
        plan.forward(f, out=g_out)
        d0 = np.random.default_rng(5100).standard_normal((geom.n_det, geom.n_t))
        dd = g_meas.clone()
        dd[0] = torch.tensor(d0, dtype=torch.float32, device=dev)
        plan.adjoint(dd, out=f_out)
        gr = g_out[0].cpu().double().numpy()[gold["det"]]
        ap = f_out[0].cpu().double().numpy().ravel()[gold["pix"]]
        parity = {"fwd_rel_l2_sampled_traces": float(np.linalg.norm(gr - gold["g_rows"]) /
                                                     np.linalg.norm(gold["g_rows"])),
                  "adj_rel_l2_sampled_pixels": float(np.linalg.norm(ap - gold["a_pix"]) /
                                                     np.linalg.norm(gold["a_pix"])),
                  "reference": "stored FP64 oracle values, tests/golden/large_1024.npz"}
        assert parity["fwd_rel_l2_sampled_traces"] <= 1e-5 and parity["adj_rel_l2_sampled_pixels"] <= 1e-5, parity
    ms_pair, _ = time_pairs(torch, plan, f, g_meas, g_out, f_out, 10, 2)
    kms = kernel_times(pat, plan, f, g_meas, g_out, f_out, 5)
    steps = args.large_steps
    rec = TVReconstructor(plan, g_meas, lam=cfg.get("tv_lambda", 1e-3))
    rec.capture(10)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rec.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ab = algorithmic_bytes(plan.info, geom, B)
    n2, dt_ = geom.n * geom.n, geom.n_det * geom.n_t
    loop_bytes = B * (8 * n2 + 16 * n2 + 12 * dt_)     # TV gradient, projected update, residual
    it_bytes = sum(ab.values()) + loop_bytes
    out = {
        "workload": "TV projected-gradient loop, 1024x1024, 1024 detectors on 270 deg, 2048 samples on (0,2], "
                    "batch %d, 1 %% noise, lambda 1e-3, HIP graphs of 10 iterations" % B,
        "iterations_per_s": round(steps * 1000.0 / ms, 2), "iterations": steps,
        "ms_per_iteration": round(ms / steps, 4),
        "pairs_per_s": round(B * 1000.0 / ms_pair, 2), "ms_per_pair_batch": round(ms_pair, 4),
        "roofline": roofline(kms, plan.info, geom, B),
        "roofline_iteration": {"bound": "hbm", "bytes_per_iteration": int(it_bytes),
                               "achieved": round(it_bytes * steps / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s",
                               "frac": round(it_bytes * steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms": {k: round(v, 4) for k, v in kms.items()},
        "parity": parity, "launch": launch, "split_batch": plan.split,
    }
    plan.close()
    return out


def bench_default(args):
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import CONFIGS, config_geometry

    dev = torch.device("cuda", 0)
    cfg = CONFIGS[2]
    geom = config_geometry(2)
    B = args.batch
    print("bench: building inputs (batch %d)" % B, file=sys.stderr, flush=True)
    plan = pat.PatPlan(geom, max_batch=B)
    plan1 = pat.PatPlan(geom, max_batch=1)
    fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, 1000)
    g_out = torch.empty_like(g_meas)
    f_out = torch.empty_like(f)
    copy_calibration(torch, dev)
    copy = measure_copy(torch, dev)
    launch = {"batched": plan.launch, "single": plan1.launch}
    if args.tune:
        print("bench: autotuning the launch shapes", file=sys.stderr, flush=True)
        launch = {"batched": plan.autotune(batch=B, cache_path=args.tune_cache),
                  "single": plan1.autotune(batch=1, cache_path=args.tune_cache)}

    print("bench: timing batched", file=sys.stderr, flush=True)
    ms_step, wall = time_pairs(torch, plan, f, g_meas, g_out, f_out, args.steps, args.warmup)
    value = B * 1000.0 / ms_step
    parity = None
    cpu = None
    if not args.no_cpu_baseline:
        # the outputs of the timed launches: g_out = A f and f_out = A* g_meas over the batch
        print("bench: oracle parity of the timed outputs + CPU baseline", file=sys.stderr, flush=True)
        idx = (0, B - 1)
        errs, t_cpu, nthreads = parity_against_oracle(np, geom, fs, gm, g_out, f_out, idx)
        parity = {"instances": errs, "fwd_rel_l2": max(e["fwd_rel_l2"] for e in errs),
                  "adj_rel_l2": max(e["adj_rel_l2"] for e in errs)}
        assert parity["fwd_rel_l2"] <= 1e-5 and parity["adj_rel_l2"] <= 1e-5, parity
        cpu = {"value": round(len(idx) / t_cpu, 4), "unit": "pairs/s", "cores": nthreads, "kind": "oracle",
               "sample": "%d x (one A + one A*): instances %s of the 256^2 batch, FP64 direct sums"
                         % (len(idx), ", ".join(str(b) for b in idx))}
    print("bench: timing single", file=sys.stderr, flush=True)
    f1, g1 = f[0:1].contiguous(), g_meas[0:1].contiguous()
    go1, fo1 = torch.empty_like(g1), torch.empty_like(f1)
    ms_single, _ = time_pairs(torch, plan1, f1, g1, go1, fo1, max(args.steps, 20), args.warmup)

    def pair1():
        plan1.forward(f1, out=go1)
        plan1.adjoint(g1, out=fo1)
    # ten pairs per graph, as the iterative workloads capture ten iterations:
    # one graph launch per ten pairs keeps the host's launch rate out of it
    ms_single_graph = time_graph(torch, dev, pair1, max(args.steps, 20), per_graph=10)
    kms = kernel_times(pat, plan, f, g_meas, g_out, f_out)
    kms1 = kernel_times(pat, plan1, f1, g1, go1, fo1)
    abytes = algorithmic_bytes(plan.info, geom, B)
    gbs = {n: abytes[n] / (kms[n] * 1e-3) / 1e9 for n in kms}
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
        # pairs (A then A*) on one instance, replayed from a HIP graph of ten pairs:
        # at batch 1 a pair is ten short kernels, and eager calls from Python time
        # the host's launch rate as much as the device (eager figures beside it)
        "single": {"value": round(1000.0 / ms_single_graph, 1), "unit": "pairs/s",
                   "ms_per_pair": round(ms_single_graph, 4), "batch": 1, "launch": "hip graph of 10 pairs",
                   "eager_value": round(1000.0 / ms_single, 1), "eager_ms_per_pair": round(ms_single, 4)},
        "batched_over_single": round(value * ms_single_graph / 1000.0, 2),
        "wall_s_timed": round(wall, 3),
        "parity": parity,
        "roofline": roofline(kms, plan.info, geom, B, copy["gbs"]),
        "roofline_step": step_roofline(kms, plan.info, geom, B, ms_step, copy["gbs"]),
        "copy_gbs": copy,
        "kernels_ms": {k: round(v, 4) for k, v in kms.items()},
        "kernels_gbs": {k: round(v, 1) for k, v in gbs.items()},
        "kernels_ms_single": {k: round(v, 4) for k, v in kms1.items()},
        "kernels_hash": kernels_hash(),
        "launch": launch, "tuned": bool(args.tune),
        # calls of at least this batch run as two half-batches on two streams (0: never)
        "split_batch": {"batched": plan.split, "single": plan1.split},
        "cpu_baseline": cpu,
    }
    plan.close()
    plan1.close()
    if not args.no_large:
        out["large"] = large_leg(args, np, torch, pat, dev)
    print(json.dumps(out), flush=True)


def bench_tv(args, cfg_id, steps_default, seed_stride):
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import TVReconstructor
    from pat_inputs import CONFIGS, config_geometry

    dev = torch.device("cuda", 0)
    cfg = CONFIGS[cfg_id]
    geom = config_geometry(cfg_id)
    B = cfg["batch"]
    steps = args.tv_steps or steps_default
    lam = cfg.get("tv_lambda", 1e-3)
    print("bench: building inputs (%dx%d, batch %d)" % (geom.n, geom.n, B), file=sys.stderr, flush=True)
    plan = pat.PatPlan(geom, max_batch=B)
    fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, seed_stride)
    if args.tune:
        plan.autotune(batch=B, cache_path=args.tune_cache)
    g_out, f_out = torch.empty_like(g_meas), torch.empty_like(f)
    ms_pair, _ = time_pairs(torch, plan, f, g_meas, g_out, f_out, 5, 2)
    gin = g_meas if B > 1 else g_meas[0]
    print("bench: TV loop, %d iterations" % steps, file=sys.stderr, flush=True)
    rec = TVReconstructor(plan, gin, lam=lam)
    rec.capture(10)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rec.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ab = algorithmic_bytes(plan.info, geom, B)
    n2, dt_ = geom.n * geom.n, geom.n_det * geom.n_t
    loop_bytes = 8 * n2 + 16 * n2 + 12 * dt_     # TV gradient, projected update, residual
    it_bytes = sum(ab.values()) + B * loop_bytes
    out = {
        "metric": "TV projected-gradient iterations/s (A, residual, A*, TV gradient, update per iteration)",
        "value": round(steps * 1000.0 / ms, 2),
        "unit": "iterations/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": round(ms / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "TV loop, %dx%d, %d detectors on %.0f deg, %d samples, batch %d, lambda %.0e, "
                               "HIP graphs of 10 iterations"
                               % (geom.n, geom.n, geom.n_det, math.degrees(geom.arc_span), geom.n_t, B, lam),
                   "batch": B},
        "staged_hbm_gbs": round(it_bytes * steps / (ms * 1e-3) / 1e9, 1),
        "pairs_per_s": round(B * 1000.0 / ms_pair, 2),
        "tau": rec.tau,
        "launch": plan.launch,
        "kernels_ms": {k: round(v, 4) for k, v in kernel_times(pat, plan, f, g_meas, g_out, f_out, 5).items()},
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_mixed(args):
    """64 heterogeneous instances (grids 128^2 / 256^2 / 512^2, 64..512
    detectors, 90 / 180 / 360 degree arcs, T = 2N): one PatBatch call per
    direction against a loop of per-instance plan calls, eager and as graphs."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import make_phantom
    from pat_inputs.geometry import mixed_batch_geometries

    dev = torch.device("cuda", 0)
    inst = mixed_batch_geometries(64)
    plans, by_geo = [], {}
    for geom, _ in inst:
        key = (geom.n, geom.n_det, geom.n_t, round(geom.arc_span, 9))
        if key not in by_geo:
            by_geo[key] = pat.PatPlan(geom)
        plans.append(by_geo[key])
    print("bench: mixed batch of %d instances, %d plans" % (len(inst), len(by_geo)), file=sys.stderr, flush=True)
    fs = [torch.tensor(make_phantom(g.n, 5, 1, 0, s), dtype=torch.float32, device=dev) for g, s in inst]
    gs = [p.forward(f) for p, f in zip(plans, fs)]
    gout = [torch.empty_like(g) for g in gs]
    aout = [torch.empty_like(f) for f in fs]
    batch = pat.PatBatch(plans)
    tuned = batch.autotune(None) if args.tune else batch.launch
    # parity: batch equals per-instance bitwise; N = 128 instances against the oracle
    bo = batch.forward(fs)
    ba = batch.adjoint(gs)
    for i, p in enumerate(plans):
        assert torch.equal(bo[i], p.forward(fs[i])) and torch.equal(ba[i], p.adjoint(gs[i])), i
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        errs = []
        for i in [i for i, (g, _) in enumerate(inst) if g.n == 128][:2]:
            g = inst[i][0]
            rf = oracle.forward(g, fs[i].cpu().double().numpy())
            ra = oracle.adjoint(g, gs[i].cpu().double().numpy())
            errs.append((float(np.linalg.norm(bo[i].cpu().double().numpy() - rf) / np.linalg.norm(rf)),
                         float(np.linalg.norm(ba[i].cpu().double().numpy() - ra) / np.linalg.norm(ra))))
        assert all(e <= 1e-5 for pair in errs for e in pair), errs
        parity = {"instances_checked": len(errs), "max_rel_l2": max(max(e) for e in errs)}

    def batched():
        batch.forward(fs, gout)
        batch.adjoint(gs, aout)

    def per_instance():
        for i, p in enumerate(plans):
            p.forward(fs[i], out=gout[i])
            p.adjoint(gs[i], out=aout[i])

    print("bench: timing", file=sys.stderr, flush=True)
    steps = max(5, args.steps // 2)
    t_b_graph = time_graph(torch, dev, batched, steps)
    t_b_eager = time_eager(torch, dev, batched, steps)
    t_p_graph = time_graph(torch, dev, per_instance, steps)
    t_p_eager = time_eager(torch, dev, per_instance, steps)
    n = len(inst)
    out = {
        "metric": "A+A* operator pairs/sec, heterogeneous batch of 64 (FP32, rel L2 <= 1e-5 vs FP64)",
        "value": round(n * 1000.0 / t_b_graph, 1), "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": round(t_b_graph, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 instances: N in {128,256,512}, D in {64,128,256,512}, arcs {90,180,360} deg, "
                               "T = 2N; one batched A and A* per step, captured as one graph",
                   "instances": n, "plans": len(by_geo)},
        "batched_graph_pairs_s": round(n * 1000.0 / t_b_graph, 1),
        "batched_eager_pairs_s": round(n * 1000.0 / t_b_eager, 1),
        "per_instance_graph_pairs_s": round(n * 1000.0 / t_p_graph, 1),
        "per_instance_eager_pairs_s": round(n * 1000.0 / t_p_eager, 1),
        "batched_over_per_instance_graph": round(t_p_graph / t_b_graph, 2),
        "batched_over_per_instance_eager": round(t_p_eager / t_b_eager, 2),
        "launch": tuned, "tuned": bool(args.tune), "parity": parity,
    }
    print(json.dumps(out), flush=True)
    batch.close()
    for p in by_geo.values():
        p.close()


def bench_pdhg(args, cfg_id, seed_stride):
    """Primal-dual TV reconstruction (the paper's classical baseline) run to the
    paper's stopping rule: relative change <= 1e-4, checked every 10 iterations."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import PDHGReconstructor
    from pat_inputs import CONFIGS, config_geometry

    dev = torch.device("cuda", 0)
    cfg = CONFIGS[cfg_id]
    geom = config_geometry(cfg_id)
    B = cfg["batch"]
    plan = pat.PatPlan(geom, max_batch=B)
    if args.sim_data:
        fs, f, gm, g_meas = make_sim_inputs(np, torch, geom, cfg, B, dev, seed_stride)
    else:
        fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, seed_stride)
    if args.tune:
        plan.autotune(batch=B, cache_path=args.tune_cache)
    alpha = 0.05 * float(np.abs(gm).max())
    gin = g_meas if B > 1 else g_meas[0]
    # untimed warm-up on a throw-away reconstructor: the run to the stopping
    # rule lasts well under a second at batch 1, short enough for clock ramp-up
    # to show in it
    n_warm = max(200, args.warmup)
    warm = PDHGReconstructor(plan, gin, alpha)
    warm.capture()
    warm.run(n_warm, tol=None)
    torch.cuda.synchronize()
    del warm
    rec = PDHGReconstructor(plan, gin, alpha)
    rec.capture()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    iters = rec.run(args.tv_steps or 5000, tol=1e-4, check_every=10)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    done = iters - 1  # the capture's warm-up iteration ran before the timed region
    rel = rec.relative_change()
    err = float(np.linalg.norm((rec.f.cpu().double().numpy() - fs).ravel()) / np.linalg.norm(fs.ravel()))
    out = {
        "metric": "primal-dual TV iterations/s (A, A*, dual and primal steps per iteration) to relative change <= 1e-4",
        "value": round(done * 1000.0 / ms, 2), "unit": "iterations/s", "n_gpus": 1, "steps": done,
        "warmup": n_warm + 1,
        "ms_per_step": round(ms / done, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic; " + ("data simulated on the %dx%d grid (FFT wave propagation), no inverse crime"
                                 % (2 * geom.n, 2 * geom.n) if args.sim_data else "data from the operator A"),
        "config": {"workload": "primal-dual TV, %dx%d, %d detectors on %.0f deg, %d samples, batch %d, "
                               "alpha = 0.05 max|g|, eta %.0f %%, stopping at relative change 1e-4 (checked every 10)"
                               % (geom.n, geom.n, geom.n_det, math.degrees(geom.arc_span), geom.n_t, B,
                                  100 * cfg["noise"]), "batch": B},
        "iterations_to_stop": iters, "seconds_to_stop": round(ms / 1000.0, 4), "wall_s": round(wall, 3),
        "final_relative_change": [round(r, 8) for r in rel],
        "rel_l2_to_phantom": round(err, 4),
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_paper(args):
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import paper_shape_geometry

    dev = torch.device("cuda", 0)
    geom = paper_shape_geometry()
    plan = pat.PatPlan(geom, max_batch=1)
    cfg = dict(phantom=(20, 3, 4), noise=0.01, seed=760)
    fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, 1, dev, 1)
    if args.tune:
        plan.autotune(batch=1, cache_path=args.tune_cache)
    g_out, f_out = torch.empty_like(g_meas), torch.empty_like(f)
    ms, _ = time_pairs(torch, plan, f, g_meas, g_out, f_out, args.steps, args.warmup)
    kms = kernel_times(pat, plan, f, g_meas, g_out, f_out, 5)
    out = {"metric": "A+A* pairs/s at the paper's timed shape",
           "value": round(1000.0 / ms, 1), "unit": "pairs/s", "ms_per_step": round(ms, 4), "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "760x760, 256 detectors on 270 deg, 2030 samples, batch 1"},
           "kernels_ms": {k: round(v, 4) for k, v in kms.items()}, "launch": plan.launch,
           "tuned": bool(args.tune)}
    print(json.dumps(out), flush=True)
    plan.close()


def bench_dense(args):
    """Explicit detector angles: the 256^2 limited-view workload with its 256
    detectors each displaced by up to +-0.3 element pitch (seeded), so the
    angular synthesis runs as the dense product on the matrix cores."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import CONFIGS
    from pat_inputs.geometry import jittered_array_geometry

    dev = torch.device("cuda", 0)
    cfg = CONFIGS[2]
    geom = jittered_array_geometry()
    B = args.batch
    plan = pat.PatPlan(geom, max_batch=B)
    fs, f, gm, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, 1000)
    g_out, f_out = torch.empty_like(g_meas), torch.empty_like(f)
    launch = plan.launch
    if args.tune:
        launch = plan.autotune(batch=B, cache_path=args.tune_cache)
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        ref_g = oracle.forward(geom, fs[0])
        ref_f = oracle.adjoint(geom, gm[0])
        g0 = plan.forward(f[0:1].contiguous())[0].cpu().double().numpy()
        a0 = plan.adjoint(g_meas[0:1].contiguous())[0].cpu().double().numpy()
        parity = {"fwd_rel_l2": float(np.linalg.norm(g0 - ref_g) / np.linalg.norm(ref_g)),
                  "adj_rel_l2": float(np.linalg.norm(a0 - ref_f) / np.linalg.norm(ref_f))}
        assert parity["fwd_rel_l2"] <= 1e-5 and parity["adj_rel_l2"] <= 1e-5, parity
    ms_step, wall = time_pairs(torch, plan, f, g_meas, g_out, f_out, args.steps, args.warmup)
    kms = kernel_times(pat, plan, f, g_meas, g_out, f_out)
    syn = {k: kms[k] for k in ("syn_fwd", "syn_adj")}
    out = {"metric": "A+A* pairs/s, explicit (jittered) detector angles, dense synthesis on the matrix cores",
           "value": round(B * 1000.0 / ms_step, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256x256, 256 detectors on 180 deg jittered by up to +-0.3 pitch, 512 samples, "
                                  "batch %d" % B, "batch": B},
           "parity": parity, "roofline": roofline(kms, plan.info, geom, B),
           "roofline_dense_synthesis": roofline(syn, plan.info, geom, B),
           "kernels_ms": {k: round(v, 4) for k, v in kms.items()}, "launch": launch, "tuned": bool(args.tune)}
    print(json.dumps(out), flush=True)
    plan.close()


def bench_cgls(args):
    """CGLS, the iterative stand-in for the fast inverse (the deep image
    prior's input): workload (2), batch B, `--tv-steps` (default 20) steps,
    two steps per HIP-graph replay."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import CGLSReconstructor
    from pat_inputs import CONFIGS, config_geometry

    dev = torch.device("cuda", 0)
    cfg, geom, B = CONFIGS[2], config_geometry(2), args.batch
    plan = pat.PatPlan(geom, max_batch=B)
    _, f, _, g_meas = make_inputs(np, torch, plan, geom, cfg, B, dev, 1000)
    launch = plan.autotune(batch=B, cache_path=args.tune_cache) if args.tune else plan.launch
    steps = args.tv_steps or 20
    steps += steps % 2
    rec = CGLSReconstructor(plan, g_meas)
    r0 = rec.residual_norm()
    rec.capture()                          # two eager steps + record two
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps // 2):
        rec.graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rn = rec.residual_norm()
    rel = float(np.max(np.asarray(rn) / np.asarray(r0)))
    out = {"metric": "CGLS steps/s (A p, A* r, two norms, two updates per step; batch of %d)" % B,
           "value": round(steps * 1000.0 / ms, 2), "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": 2,
           "ms_per_step": round(ms / steps, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "CGLS, limited-view 256x256, 256 detectors on 180 deg, 512 samples, batch %d, "
                                  "two steps per HIP graph" % B, "batch": B},
           "relative_residual_after": round(rel, 5), "launch": launch, "tuned": bool(args.tune)}
    print(json.dumps(out), flush=True)
    plan.close()


def bench_dip(args):
    """Deep image prior (eq. (5)) at the paper's timed shape: U-Net forward and
    backward (float32, stock layers), A and A* in this library's kernels, the
    TV kernel, an Adam step; the input z from 10 CGLS steps."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.dip import DIPReconstructor
    from paper_2604_19176_amd.recon import CGLSReconstructor
    from pat_inputs import paper_shape_geometry

    dev = torch.device("cuda", 0)
    geom = paper_shape_geometry()
    plan = pat.PatPlan(geom, max_batch=1)
    cfg = dict(phantom=(20, 3, 4), noise=0.01, seed=760)
    _, f, _, g_meas = make_inputs(np, torch, plan, geom, cfg, 1, dev, 1)
    g1 = g_meas[0].contiguous()
    launch = plan.autotune(batch=1, cache_path=args.tune_cache) if args.tune else plan.launch
    cg = CGLSReconstructor(plan, g1)
    for _ in range(10):
        cg.step()
    steps = args.steps
    rec = DIPReconstructor(plan, g1, cg.f, lam=0.1, iters=steps + args.warmup)
    for _ in range(args.warmup):
        rec.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        rec.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gout, fout = torch.empty_like(g1), torch.empty_like(f[0])
    kms = kernel_times(pat, plan, f[0].contiguous(), g1, gout, fout, 5)
    op_ms = sum(kms.values())
    out = {"metric": "DIP iterations/s at the paper's timed shape (U-Net fwd+bwd, A, A*, TV, Adam)",
           "value": round(1000.0 / ms, 2), "unit": "iterations/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "DIP, 760x760, 256 detectors on 270 deg, 2030 samples, batch 1, U-Net 32-256 "
                                  "channels", "batch": 1},
           "operator_pair_ms": round(op_ms, 4), "operator_share": round(op_ms / ms, 4),
           "paper_context": "142.9 ms per DIP iteration on an RTX A5000 (Sec. 4.3; other hardware)",
           "final_objective": float(rec.last_loss), "launch": launch, "tuned": bool(args.tune)}
    print(json.dumps(out), flush=True)
    plan.close()


def bench_sim(args):
    """The wave-propagation data simulator at the simulation study's shape:
    512^2 fine grid, 256 detectors on 270 deg, 512 samples on (0, 2]."""
    import numpy as np
    import torch

    import paper_2604_19176_amd as pat
    from pat_inputs import Geometry, make_phantom

    dev = torch.device("cuda", 0)
    geom = Geometry(n=512, n_det=256, n_t=512, dt=2.0 / 512, arc_span=math.radians(270.0))
    f_np = make_phantom(geom.n, 20, 3, 4, 512)
    f = torch.tensor(f_np, dtype=torch.float32, device=dev)
    sim = pat.PatSim(geom)
    g = torch.empty((geom.n_det, geom.n_t), dtype=torch.float32, device=dev)
    steps = max(1, min(args.steps, 20))
    for _ in range(max(1, args.warmup)):
        sim.run(f, out=g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        sim.run(f, out=g)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    M = sim.box_side
    pairs = (geom.n_t + 1) // 2
    parity, cpu = None, None
    if not args.no_cpu_baseline:
        from oracle import simulate as ref
        cols = [0, 255, 511]
        t0 = time.perf_counter()
        g_ref = ref.simulate(geom, f_np, times=[(j + 1) * geom.dt for j in cols])
        t_cpu = time.perf_counter() - t0
        gg = g.cpu().double().numpy()[:, cols]
        parity = {"sampled_times": cols,
                  "rel_l2": float(np.linalg.norm(gg - g_ref) / np.linalg.norm(g_ref))}
        cpu = {"seconds_per_time_sample": round(t_cpu / len(cols), 4), "kind": "oracle (numpy FP64 FFTs)",
               "sample": "3 time samples of the same simulation"}
    out = {"metric": "wave-propagation simulations/s (FFT k-space propagator on the fine grid, Keys sampling)",
           "value": round(1000.0 / ms, 2), "unit": "simulations/s", "ms_per_step": round(ms, 4), "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "simulator: 512x512 fine grid (box %d), 256 detectors on 270 deg, "
                                  "512 samples on (0,2]" % M, "box": M},
           # per simulation: the box spectrum is read once per pair of samples by the column pass
           "bytes_spectrum_reads_per_simulation": int(8 * M * M * pairs),
           "parity": parity, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    sim.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", default="default",
                    choices=["default", "mixed", "tv3", "large", "paper", "pdhg3", "pdhg-large", "dense", "cgls",
                             "dip", "sim"])
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="time the default launch shapes instead of autotuning them first")
    ap.add_argument("--tune-cache", default=None, help="JSON cache file of the autotuner")
    ap.add_argument("--tv-steps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="default workload: skip the 1024^2 TV leg (the 'large' key of the line)")
    ap.add_argument("--large-steps", type=int, default=2000,
                    help="TV iterations of the 1024^2 leg of the default workload")
    ap.add_argument("--sim-data", action="store_true",
                    help="pdhg workloads: measurements from the data simulator on a twice finer grid")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the operator pair shards by instance with no "
              "communication, so --gpus %d is not run" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "default":
        bench_default(args)
    elif args.workload == "dip":
        bench_dip(args)
    elif args.workload == "cgls":
        bench_cgls(args)
    elif args.workload == "dense":
        bench_dense(args)
    elif args.workload == "mixed":
        bench_mixed(args)
    elif args.workload == "pdhg3":
        bench_pdhg(args, 3, 1000)
    elif args.workload == "pdhg-large":
        bench_pdhg(args, 5, 1)
    elif args.workload == "tv3":
        bench_tv(args, 3, 500, 1000)
    elif args.workload == "large":
        bench_tv(args, 5, 2000, 1)
    elif args.workload == "sim":
        bench_sim(args)
    else:
        bench_paper(args)


if __name__ == "__main__":
    main()
