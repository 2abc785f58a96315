"""Throughput of the 3rd-RF horizontal covariance operator V_H and its adjoint on one MI355X.

Step = one forward application V_H x (G_y G_x) plus one adjoint application
V_H^T x (G_x^T G_y^T) of the FP32 3rd-RF on the global quarter-degree-shaped
workload: 1440 x 720 grid, 50 levels, ~30% land, sigma = 1.5 + 10.5 cos^2(lat)
grid points, 4 imaginary points per coast, fitted q(sigma).  Inputs are
resident in device memory before the timed region; the coefficient block is
built once (setup, outside the timed region, as in the paper's scheme where
coefficients depend only on the grid).

Prints ONE JSON line.  Extra keys: per-direction kernel times, the FP64 1st-RF
(K = 5) baseline on the same grid and the speedup of the FP32 3rd-RF forward
over it, and the FP64 CPU oracle timed on a sample of levels.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoints/s of 3rd-RF fwd+adjoint (FP32 batched vs FP64 1st-RF) and % HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1404_5756_amd", "csrc", "sweep_fast.hip")


def kernel_code_hash(path=KERNEL_SRC):
    """sha256 of the kernel source without comments and blank space: the traffic
    figures stay valid across comment-only edits, not across code changes."""
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = "\n".join(" ".join(line.split()) for line in src.splitlines() if line.strip())
    return hashlib.sha256(src.encode()).hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bench_batch(torch, dev, args):
    """64 uneven grids (C4) in one batch: forward + adjoint, against one call per grid.
    The work-list shape is autotuned on the items; the tuned batch is also timed as
    hipGraph replays of one captured forward + adjoint."""
    from paper_1404_5756_amd import synth
    from paper_1404_5756_amd.operator import Batch, HorizontalCovariance
    ws = synth.c4_batch()
    gen = torch.Generator(device=dev).manual_seed(synth.SEEDS["c4"])
    t0 = time.time()
    ops, xs, ys = [], [], []
    for w in ws:
        ops.append(HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode,
                                        device=dev))
        xs.append(torch.randn((1, w.nlev, w.ny, w.nx), generator=gen, device=dev))
        ys.append(torch.empty_like(xs[-1]))
    b = Batch([(op, x, y) for op, x, y in zip(ops, xs, ys)])
    torch.cuda.synchronize()
    setup = time.time() - t0
    pts = b.points
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(3, args.steps // 4)
    ms_i = timed(lambda: [(op.apply(x, out=y), op.adjoint(x, out=y)) for op, x, y in zip(ops, xs, ys)], reps)
    t1 = time.time()
    tune_times = b.autotune(reps=2)
    tune_s = time.time() - t1
    # default and tuned shapes in alternating rounds, after tuning (same clocks)
    b0 = Batch([(op, x, y) for op, x, y in zip(ops, xs, ys)])
    ms_default = ms_tuned = 0.0
    for _ in range(3):
        ms_default += timed(lambda: (b0.apply(False), b0.apply(True)), reps) / 3
        ms_tuned += timed(lambda: (b.apply(False), b.apply(True)), reps) / 3
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.apply(False)
        b.apply(True)
    ms_graph = timed(g.replay, max(reps, 10))
    ms_b = min(ms_tuned, ms_graph)
    log(f"batch C4: {len(ws)} grids, {pts / 1e9:.3f} G points: fwd+adj default shape {ms_default:.2f} ms, "
        f"autotuned {b.tuning} {ms_tuned:.2f} ms, graph replay {ms_graph:.2f} ms; per-grid calls {ms_i:.2f} ms "
        f"(setup {setup:.1f} s, autotune {tune_s:.1f} s over {len(tune_times)} shapes)")
    res = {"grids": len(ws), "points": pts, "ms_fwd_adj": round(ms_b, 3),
           "gpoints_s": round(pts / (ms_b * 1e-3) / 1e9, 2), "ms_default_shape": round(ms_default, 3),
           "ms_autotuned": round(ms_tuned, 3), "ms_graph_replay": round(ms_graph, 3),
           "tuning": {"x_groups_max": b.tuning[0], "y_planes": b.tuning[1], "x_one_launch": b.tuning[2]}
           if b.tuning else "default",
           "ms_per_grid_calls": round(ms_i, 3), "speedup_vs_per_grid_calls": round(ms_i / ms_b, 3),
           "setup_s": round(setup, 1), "autotune_s": round(tune_s, 1)}
    del g, b, ops, xs, ys
    torch.cuda.empty_cache()
    return res


def k_frontier(torch, dev, w, x, ms_rf3_fwd, args):
    """Accuracy/time frontier of the 1st-RF over K against the 3rd-RF (the GPU analogue of the
    paper's K = 1, 5, 10 comparison): time of the fused FP32 1st-RF on the workload for each K, and
    the Gaussian shape error of the GPU impulse response on an all-sea line (sigma = 4 and 12):
    || h/sum h - g/sum g || / || g/sum g || with g the Gaussian of width sigma."""
    from paper_1404_5756_amd.operator import HorizontalCovariance
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.empty_like(x)

    def shape_err(sig, K=None):
        n = int(60 * sig) | 1
        mask = np.ones((1, 1, n), np.uint8)
        s = np.full((1, 1, n), float(sig))
        op1 = HorizontalCovariance(mask, s, s, 1, n_img=0, qmode="fit", k1=K or 1, device=dev)
        imp = torch.zeros((1, 1, n), dtype=torch.float64, device=dev)
        imp[0, 0, n // 2] = 1.0
        h = (op1.rf1_fused(imp, K=K) if K else op1.apply_dir(imp, "x")).cpu().numpy().ravel()
        i = np.arange(n) - n // 2
        g = np.exp(-i * i / (2.0 * sig * sig))
        hn, gn = h / h.sum(), g / g.sum()
        return float(np.linalg.norm(hn - gn) / np.linalg.norm(gn))

    res = {"rf3_fit": {"ms_fwd": round(ms_rf3_fwd, 4), "shape_err_sigma4": round(shape_err(4.0), 4),
                       "shape_err_sigma12": round(shape_err(12.0), 4)}}
    for K in (1, 2, 3, 5, 10):
        op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=K,
                                  device=dev)
        op.rf1_fused(x, K=K, out=out)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            op.rf1_fused(x, K=K, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        res[f"rf1_k{K}"] = {"ms_fused_fp32": round(ms, 4), "shape_err_sigma4": round(shape_err(4.0, K), 4),
                            "shape_err_sigma12": round(shape_err(12.0, K), 4)}
        del op
    log("K frontier: " + ", ".join(f"{k} {v}" for k, v in res.items()))
    return res


def bench_variants(torch, dev, args):
    """C3 step (forward + adjoint) with the options beyond the paper's scheme: zonally periodic
    rows, exact end conditions, anisotropic inhomogeneous length scales, and a depth-dependent
    mask and sigma (per-level tables) (same field); and C2 (T and S, 72 levels) with a
    depth-dependent mask and sigma (its own two-field input)."""
    from paper_1404_5756_amd import synth
    from paper_1404_5756_amd.operator import HorizontalCovariance
    res = {}
    base = synth.c3_global()
    x = torch.from_numpy(base.field(np.float32)).to(dev)
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, w, kw in (("periodic_x", base, {"periodic_x": True}), ("exact_ends", base, {"exact_ends": True}),
                        ("anisotropic", synth.c3_anisotropic(), {}), ("depth_mask_sigma", synth.c3_depth(), {}),
                        ("c2_depth_TS", synth.c2_depth(), {})):
        if w.points != base.points:
            x = torch.from_numpy(w.field(np.float32)).to(dev)
            out = torch.empty_like(x)
        op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, device=dev,
                                  **kw)
        for _ in range(5):
            op.apply(x, out=out)
            op.adjoint(x, out=out)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            op.apply(x, out=out)
            op.adjoint(x, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = {"ms_fwd_adj": round(ms, 4), "gpoints_s": round(w.points / (ms * 1e-3) / 1e9, 2)}
        log(f"variant {name}: fwd+adj {ms:.3f} ms -> {res[name]['gpoints_s']} Gpoints/s")
        del op
    torch.cuda.empty_cache()
    return res


def bench_cg(torch, dev, w, op, args):
    """3D-VAR CG iterations (C5) on the C3 grid with 200k bilinear observations, FP32."""
    from paper_1404_5756_amd.var3d import synthetic_problem
    t0 = time.time()
    prob, _vt = synthetic_problem(w, 200_000, dev, torch.float32, op=op)
    torch.cuda.synchronize()
    setup = time.time() - t0
    prob.cg(1, track_cost=False)   # warm up
    torch.cuda.synchronize()
    # iterations alone (V, H, H^T, V^T and the CG vector updates; J is evaluated only at both ends)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    _v, ends = prob.cg(args.cg_iters, track_cost=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    # a second run with J after every iteration checks that J never increases
    _v2, costs = prob.cg(args.cg_iters)
    log(f"CG C5: {args.cg_iters} iterations in {ms_total:.1f} ms (incl. J at both ends); "
        f"J {costs[0]:.4e} -> {costs[-1]:.4e}")
    return {"iterations": args.cg_iters, "ms_per_iteration": round(ms_total / args.cg_iters, 3),
            "obs": 200_000, "J_first": costs[0], "J_last": costs[-1],
            "J_monotone": bool(all(c1 <= c0 * (1 + 1e-6) for c0, c1 in zip(costs, costs[1:]))),
            "setup_s": round(setup, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2"])
    ap.add_argument("--cpu-levels", type=int, default=0,
                    help="levels of the workload the CPU oracle runs on (0 = all levels)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rf1", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-grid batch (C4)")
    ap.add_argument("--no-cg", action="store_true", help="skip the 3D-VAR CG iterations (C5)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the periodic / exact-end / anisotropic C3 variants")
    ap.add_argument("--cg-iters", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); every (field, level) is an "
              "independent V_H application, so N GPUs would shard levels with no communication.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1404_5756_amd import synth
    from paper_1404_5756_amd.operator import HorizontalCovariance

    dev = torch.device("cuda:0")
    w = synth.c3_global() if args.workload == "c3" else synth.c2_regional()
    log(f"workload {w.name}: {w.nx}x{w.ny}x{w.nlev} x {w.nfields} fields, {w.points / 1e6:.2f} M points")
    t0 = time.time()
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode, k1=5,
                              device=dev)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    x_host = w.field(np.float32)
    x = torch.from_numpy(x_host).to(dev)
    out_f = torch.empty_like(x)
    out_a = torch.empty_like(x)
    pts = w.points
    stream = torch.cuda.current_stream()

    # ---- per-kernel times, in the step's own order and data flow (rf3_apply_xy is
    # x: x -> out then y: out -> out; rf3_adjoint_xy is y then x), one event between
    # launches; each call of rf3_apply_dir is one kernel launch
    reps = max(5, args.steps)
    seq = (("x_fwd", 0, False, x, out_f), ("y_fwd", 1, False, out_f, out_f),
           ("y_adj", 1, True, x, out_a), ("x_adj", 0, True, out_a, out_a))
    # its own warm-up (the GPU's clocks settle over the first ~100 ms of work)
    for _ in range(max(50, reps)):
        for name, d, adj, src, dst in seq:
            op.apply_dir(src, d, adj, out=dst)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(seq) + 1)] for _ in range(reps)]
    for r in range(reps):
        evs[r][0].record(stream)
        for k, (name, d, adj, src, dst) in enumerate(seq):
            op.apply_dir(src, d, adj, out=dst)
            evs[r][k + 1].record(stream)
    torch.cuda.synchronize()
    kern = {name: sum(evs[r][k].elapsed_time(evs[r][k + 1]) for r in range(reps)) / reps
            for k, (name, *_rest) in enumerate(seq)}
    log("kernel ms: " + ", ".join(f"{k} {v:.3f}" for k, v in kern.items()))
    # the same launches with the last-level (Infinity) cache flushed before each one:
    # 1 GiB written between launches evicts the 256 MB MALL, so the kernel reads its
    # field and tables from HBM (the in-step times above can be partly cache-served)
    flush = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(len(seq))]
    kern_flushed = {name: 0.0 for name, *_r in seq}
    freps = max(3, reps // 5)
    for r in range(freps):
        for k, (name, d, adj, src, dst) in enumerate(seq):
            flush.fill_(float(r + k))
            ev2[k][0].record(stream)
            op.apply_dir(src, d, adj, out=dst)
            ev2[k][1].record(stream)
        torch.cuda.synchronize()
        for k, (name, *_r) in enumerate(seq):
            kern_flushed[name] += ev2[k][0].elapsed_time(ev2[k][1]) / freps
    del flush
    torch.cuda.empty_cache()
    log("kernel ms, cache flushed between launches: " + ", ".join(f"{k} {v:.3f}" for k, v in kern_flushed.items()))
    # ---- the step: forward + adjoint
    for _ in range(args.warmup):
        op.apply(x, out=out_f)
        op.adjoint(x, out=out_a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        op.apply(x, out=out_f)
        op.adjoint(x, out=out_a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    value = pts / (ms_step * 1e-3) / 1e9
    log(f"step (fwd+adj): {ms_step:.3f} ms -> {value:.1f} Gpoints/s")

    dom = max(kern, key=kern.get)
    bytes_per_launch = 8.0 * pts        # FP32 read + write of every point once
    achieved = bytes_per_launch / (kern[dom] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        # '#' lines are commentary; the rest is one JSON object written from rocprofv3 counters
        tf = json.loads("".join(l for l in open(TRAFFIC_FILE) if not l.lstrip().startswith("#")))
        src_hash = kernel_code_hash()
        if tf.get("kernel_code_sha256") == src_hash and dom in tf.get("bytes_per_launch", {}):
            traffic = tf["bytes_per_launch"][dom]
    achieved_flushed = bytes_per_launch / (kern_flushed[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "achieved_cache_flushed": round(achieved_flushed, 1),
                "frac_cache_flushed": round(achieved_flushed / HBM_PEAK_GBS, 4)}
    step_frac = 4 * bytes_per_launch / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    # ---- forward alone and the FP64 1st-RF baseline (K = 5), same grid and field
    e0.record(stream)
    for _ in range(reps):
        op.apply(x, out=out_f)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / reps
    rf1 = None
    if not args.no_rf1:
        x64 = x.double()
        o64 = torch.empty_like(x64)
        op.rf1(x64, K=5, out=o64)
        torch.cuda.synchronize()
        r1reps = 3
        e0.record(stream)
        for _ in range(r1reps):
            op.rf1(x64, K=5, out=o64)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_rf1 = e0.elapsed_time(e1) / r1reps
        # fused 1st-RF: all K iterations of a direction on chip (FP64 and FP32)
        def timed_rf1(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps
        ms_f64 = timed_rf1(lambda: op.rf1_fused(x64, K=5, out=o64))
        o32 = torch.empty_like(x)
        ms_f32 = timed_rf1(lambda: op.rf1_fused(x, K=5, out=o32))
        # the FP64 3rd-RF (line-sequential kernels, the printed form), forward + adjoint
        ms_rf3_64 = timed_rf1(lambda: (op.apply(x64, out=o64), op.adjoint(x64, out=o64)), 3)
        rf1 = {"ms": round(ms_rf1, 3), "gpoints_s": round(pts / (ms_rf1 * 1e-3) / 1e9, 2),
               "speedup_rf3_fp32_fwd_vs_rf1_fp64_k5": round(ms_rf1 / ms_fwd, 2),
               "fused_fp64_ms": round(ms_f64, 3), "speedup_rf3_fp32_fwd_vs_fused_rf1_fp64_k5": round(ms_f64 / ms_fwd, 2),
               "fused_fp32_ms": round(ms_f32, 3), "speedup_rf3_fp32_fwd_vs_fused_rf1_fp32_k5": round(ms_f32 / ms_fwd, 2),
               "rf3_fp64_fwd_adj_ms": round(ms_rf3_64, 3)}
        log(f"1st-RF K=5: plain FP64 {ms_rf1:.3f} ms, fused FP64 {ms_f64:.3f} ms, fused FP32 {ms_f32:.3f} ms; "
            f"3rd-RF FP32 forward {ms_fwd:.3f} ms; 3rd-RF FP64 forward + adjoint {ms_rf3_64:.3f} ms")
        rf1["k_frontier"] = k_frontier(torch, dev, w, x, ms_fwd, args)
        del x64, o64, o32

    # ---- a plain copy of the field (known bytes): the reference that scales the
    # FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 run of this script
    out_f.copy_(x)
    torch.cuda.synchronize()

    variants = None if args.no_variants else bench_variants(torch, dev, args)
    batch = None if args.no_batch else bench_batch(torch, dev, args)
    cg = None if args.no_cg else bench_cg(torch, dev, w, op, args)

    # ---- CPU oracle baseline on a sample of levels, and parity on that sample
    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle
        oracle.build()
        nl = w.nlev if args.cpu_levels <= 0 else max(1, min(args.cpu_levels, w.nlev))
        P = oracle.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=oracle.QMODES[w.qmode], k1=5)
        xs = x_host[:1, :nl].astype(np.float64)
        threads = os.cpu_count() or 1
        times = []
        for _rep in range(3):   # median of three runs of the sample
            t0 = time.time()
            ref_f = P.rf3(xs, threads=threads)
            ref_a = P.rf3_adjoint(xs, threads=threads)
            times.append(time.time() - t0)
        cpu_s = sorted(times)[1]
        sample_pts = w.nx * w.ny * nl
        cpu = {"value": round(sample_pts / (cpu_s / 1.0) / 1e9, 5), "unit": "Gpoints/s", "cores": threads,
               "kind": "oracle", "seconds": round(cpu_s, 2),
               "sample": f"fwd+adj V_H of {nl} of {w.nlev} levels ({sample_pts / 1e6:.2f} M points), FP64 C oracle, "
                         f"OpenMP over lines, median of 3 runs"}
        # the same oracle on one thread, on 5 levels
        n1 = min(5, nl)
        t0 = time.time()
        P.rf3(xs[:, :n1], threads=1)
        P.rf3_adjoint(xs[:, :n1], threads=1)
        t1s = time.time() - t0
        cpu["one_thread"] = {"value": round(w.nx * w.ny * n1 / t1s / 1e9, 5), "unit": "Gpoints/s",
                             "seconds": round(t1s, 2), "sample": f"fwd+adj V_H of {n1} levels, 1 thread"}
        log(f"cpu oracle on 1 thread: {t1s:.2f} s for {n1} levels")
        # the oracle's plain 1st-RF (K = 5) on the same sample, and the oracle's 3rd-RF on C2 (T and S)
        t0 = time.time()
        P.rf1(xs, K=5, threads=threads)
        t_rf1 = time.time() - t0
        cpu["rf1_k5"] = {"value": round(sample_pts / t_rf1 / 1e9, 5), "unit": "Gpoints/s", "seconds": round(t_rf1, 2),
                         "sample": f"1st-RF K = 5, x then y, of {nl} levels, {threads} threads"}
        from paper_1404_5756_amd import synth
        w2 = synth.c2_regional()
        P2 = oracle.Problem(w2.mask, w2.sigma_x, w2.sigma_y, n_img=w2.n_img, qmode=oracle.QMODES[w2.qmode], k1=5)
        x2 = w2.field(np.float64)
        t0 = time.time()
        P2.rf3(x2, threads=threads)
        P2.rf3_adjoint(x2, threads=threads)
        t_c2 = time.time() - t0
        cpu["c2"] = {"value": round(w2.points / t_c2 / 1e9, 5), "unit": "Gpoints/s", "seconds": round(t_c2, 2),
                     "sample": f"fwd+adj V_H of C2 (871 x 253 x 72, T and S), {threads} threads"}
        # one oracle CG iteration of C5 (the C3 grid, 200k observations), after the initial residual
        import oracle.var3d as ov
        lev, ox, oy = synth.c5_observations(w)
        idx, wt = ov.obs_weights(w.nx, w.ny, lev, ox, oy)
        shape = (1, w.nlev, w.ny, w.nx)
        n = int(np.prod(shape))
        yobs = np.random.default_rng(5).standard_normal(len(lev))
        t0 = time.time()
        ov.cg(lambda v: P.rf3(v.reshape(shape), threads=threads).ravel(),
              lambda v: P.rf3_adjoint(v.reshape(shape), threads=threads).ravel(), idx, wt, yobs, 4.0, n, 0)
        t_r0 = time.time() - t0
        t0 = time.time()
        ov.cg(lambda v: P.rf3(v.reshape(shape), threads=threads).ravel(),
              lambda v: P.rf3_adjoint(v.reshape(shape), threads=threads).ravel(), idx, wt, yobs, 4.0, n, 1)
        t_it = time.time() - t0 - t_r0
        cpu["c5_cg_iteration"] = {"seconds": round(t_it, 2),
                                  "sample": f"one CG iteration (V, H, H^T, V^T, vector updates) of C5, {threads} threads"}
        log(f"cpu oracle: 1st-RF K=5 {t_rf1:.2f} s for {nl} levels; C2 fwd+adj {t_c2:.2f} s; "
            f"one C5 CG iteration {t_it:.2f} s")
        del x2, P2
        op.apply(x, out=out_f)
        op.adjoint(x, out=out_a)
        torch.cuda.synchronize()
        gf = out_f[:1, :nl].double().cpu().numpy()
        ga = out_a[:1, :nl].double().cpu().numpy()
        parity = {"levels": nl,
                  "fwd_rel_l2": float(np.linalg.norm(gf - ref_f) / np.linalg.norm(ref_f)),
                  "adj_rel_l2": float(np.linalg.norm(ga - ref_a) / np.linalg.norm(ref_a)), "tol": 1e-5}
        log(f"cpu oracle: {cpu_s:.2f} s on {threads} threads; parity {parity}")

    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: fwd+adjoint V_H, FP32, {w.nx}x{w.ny} grid x {w.nlev} levels x "
                               f"{w.nfields} field, n_img={w.n_img}, q={w.qmode}", "points": pts,
                   "step": "rf3_apply_xy + rf3_adjoint_xy", "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_frac_step": round(step_frac, 4),
        "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "kernel_ms_cache_flushed": {k: round(v, 4) for k, v in kern_flushed.items()},
        "rf3_fwd_ms": round(ms_fwd, 4),
        "rf1_fp64_k5": rf1,
        "c3_variants": variants,
        "batch_c4": batch,
        "cg_c5": cg,
        "parity_sample": parity,
        "setup_s": round(setup_s, 2),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
