"""Benchmark: calibrated visibilities/s of the per-interval gain solver on one MI355X.

Workload (one GPU): MeerKAT-shaped full-Jones solve: 64 antennas (2016
baselines), 600 times x 1024 channels (856-1712 MHz), complex64 data and model
from 20 point sources, complex-2x2 truth gains smooth in time and frequency
with leakage, 10% flags, noise sigma 0.05 with weights 1/sigma^2, solution
interval 1 time x 64 channels (9600 intervals of 129,024 samples).  Inputs are
seeded synthetic stand-ins for the paper's MeerKAT observation and are resident
in HBM before timing starts.

One step = solve the complex-2x2 term on every interval from unit gains to
tol 1e-6 (max 100 updates, MIXED precision: complex64 products, FP32
compensated sums, FP64 block solves) + one residual pass over all samples.
value = samples / step time.  The dominant kernel (the fused solve) is timed
with HIP events on its launch stream; its algorithmic bytes are
sum over intervals of (passes x (samples x 81 B + rows x 12 B)).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SAMPLE = 32 + 32 + 16 + 1        # data c64 2x2, model c64 2x2, 4 fp32 weights, 1 flag byte
BYTES_PER_ROW = 12                          # ant1, ant2, row_time int32


# FP32 arithmetic of the full-Jones solver step per sample and pass, counted in
# the ISA of the single-term kernel: 200 fused multiply-adds (2 flop) and 40
# multiplies
FLOP_PER_SAMPLE_C2X2 = 2 * 200 + 40


def interval_samples(vis, term_h):
    """Samples (rows x channels) of each solution interval of a term, [n_gt][n_gf]."""
    import numpy as np
    t_map = np.asarray(term_h.t_map.cpu() if hasattr(term_h.t_map, "cpu") else term_h.t_map)
    f_map = np.asarray(term_h.f_map.cpu() if hasattr(term_h.f_map, "cpu") else term_h.f_map)
    rows = np.bincount(t_map[vis.row_time.cpu().numpy()], minlength=int(term_h.n_gt)).astype(np.float64)
    chans = np.bincount(f_map, minlength=int(term_h.n_gf)).astype(np.float64)
    return rows[:, None] * chans[None, :]


def copy_bandwidth(dev, n_bytes: int = 1 << 32, reps: int = 5) -> float:
    """Device-to-device copy of n_bytes (read + write counted), best of reps, GB/s:
    the streaming rate this GPU sustains, beside the nominal HBM peak."""
    import torch
    src = torch.empty(n_bytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n_bytes / (best * 1e-3) / 1e9


def pass_bytes(vis, term_h):
    """Algorithmic HBM bytes of one solver pass over each solution interval of a
    term, [n_gt][n_gf]: samples x (data + model over every direction + weights +
    flag) + rows x row metadata (read once per 64-channel chunk)."""
    import numpy as np
    elt = vis.data.element_size()                           # one complex correlation
    per_sample = 4 * elt * (1 + int(vis.model.shape[2])) + int(vis.weight.shape[2]) * vis.weight.element_size() + 1
    t_map = np.asarray(term_h.t_map.cpu() if hasattr(term_h.t_map, "cpu") else term_h.t_map)
    f_map = np.asarray(term_h.f_map.cpu() if hasattr(term_h.f_map, "cpu") else term_h.f_map)
    rows = np.bincount(t_map[vis.row_time.cpu().numpy()], minlength=int(term_h.n_gt)).astype(np.float64)
    chans = np.bincount(f_map, minlength=int(term_h.n_gf)).astype(np.float64)
    return rows[:, None] * chans[None, :] * per_sample + rows[:, None] * BYTES_PER_ROW * np.ceil(chans[None, :] / 64.0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources the main line's solve kernel is built from: the traffic record holds
# their hash, and a change to any of them retires the record.
TRAFFIC_SOURCES = [
    "include/qc.h",
    "paper_2412_10072_amd/csrc/qc_internal.h",
    "paper_2412_10072_amd/csrc/qc_interval.h",
    "paper_2412_10072_amd/csrc/qc_band.h",
    "paper_2412_10072_amd/csrc/qc_solve_kernels.h",
    "paper_2412_10072_amd/csrc/qc_solve_kc2x2_mixed.hip",
]
TRAFFIC_RECORD = os.path.join("profiles", "k_solve_fused_meerkat_fulljones_traffic.json")


def write_traffic_record(fetch_dir: str, write_dir: str, algorithmic_bytes: float):
    """The traffic record from two rocprofv3 --pmc runs of `bench.py --legs none --steps 1 --warmup 0
    --no-cpu-baseline --calib-copy` (FETCH_SIZE in fetch_dir, WRITE_SIZE in write_dir, csv output):
    the main line's solve dispatch, scaled by what the same counters read for the 4 GiB
    calibration copy (its largest copy dispatch)."""
    import csv
    import glob
    import hashlib

    def per_dispatch(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], r["Dispatch_Id"])
                vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
        return vals

    def pick(vals, pattern):
        hits = [v for (k, _), v in vals.items() if pattern in k]
        return hits

    fetch = per_dispatch(fetch_dir, "FETCH_SIZE")
    write = per_dispatch(write_dir, "WRITE_SIZE")
    kern = "k_solve_fused<1, float, float, 1, 1, 4, false, false>"
    f_solve, w_solve = pick(fetch, kern), pick(write, kern)
    f_copy, w_copy = max(pick(fetch, "copyBuffer")), max(pick(write, "copyBuffer"))
    if len(f_solve) != 1 or len(w_solve) != 1:
        raise SystemExit(f"expected one solve dispatch per run, found {len(f_solve)} and {len(w_solve)}")
    copy_bytes = 1 << 32
    fetch_scale = copy_bytes / (f_copy * 1024.0)
    write_scale = copy_bytes / (w_copy * 1024.0)
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    fb = f_solve[0] * 1024.0 * fetch_scale
    wb = w_solve[0] * 1024.0 * write_scale
    rec = {"kernel": kern, "workload": "MeerKAT-shaped full-Jones solve, 64 ants, 600 x 1024, tol 1e-6",
           "sources": TRAFFIC_SOURCES, "sources_sha256": h.hexdigest(),
           "fetch_size_kib": f_solve[0], "write_size_kib": w_solve[0], "calib_copy_bytes": copy_bytes,
           "calib_fetch_kib": f_copy, "calib_write_kib": w_copy, "fetch_scale": fetch_scale,
           "write_scale": write_scale, "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb,
           "algorithmic_bytes": algorithmic_bytes}
    with open(os.path.join(ROOT, TRAFFIC_RECORD), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"traffic record: {fb / 1e9:.1f} GB fetched + {wb / 1e9:.3f} GB written = "
          f"{(fb + wb) / algorithmic_bytes:.3f} x the algorithmic bytes")


def measured_traffic():
    """HBM bytes per launch of the solve kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (calibrated on a copy of known size), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, TRAFFIC_RECORD)
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


def _one_blas_thread():
    """Pool worker start-up: one BLAS thread per process (the pool supplies the parallelism)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _noop(_):
    return 0


def _oracle_interval(task):
    """Pool worker: one interval solved to tol 1e-6 by the oracle; returns its samples."""
    from oracle import solver as o_solver
    vis_k, term_k = task
    o_solver.solve_term(vis_k, [term_k], 0, tol=1e-6, max_iter=100)
    return int(vis_k.data.shape[0]) * int(vis_k.data.shape[1])


def cpu_baseline_pool(prob, n_times: int = 4, workers: int = 0):
    """The oracle over a pool of host processes (one interval per task, one BLAS
    thread each): the intervals of the first n_times times, timed from the
    first task to the last result, the workers started beforehand."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    from synth.generate import slice_times, to_numpy_vis
    workers = workers or min(16, os.cpu_count() or 1)
    term = prob.chain[0]
    f_map = np.asarray(term.f_map)
    tasks = []
    for t in range(n_times):
        vis_h = to_numpy_vis(slice_times(prob.vis, t, t + 1))
        for gf in range(int(term.n_gf)):
            ch = np.nonzero(f_map == gf)[0]
            vis_k = vis_h.copy(data=np.ascontiguousarray(vis_h.data[:, ch]),
                               model=np.ascontiguousarray(vis_h.model[:, ch]),
                               weight=np.ascontiguousarray(vis_h.weight[:, ch]),
                               flag=np.ascontiguousarray(vis_h.flag[:, ch]), chan_freq=vis_h.chan_freq[ch])
            term_k = term.copy(t_map=np.zeros(1, np.int32), f_map=np.zeros(ch.size, np.int32), n_gt=1, n_gf=1,
                               gains=term.gains[:1, :1].copy(), gain_flags=term.gain_flags[:1, :1].copy())
            tasks.append((vis_k, term_k))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                             initializer=_one_blas_thread) as ex:
        list(ex.map(_noop, range(4 * workers)))
        t0 = time.perf_counter()
        samples = sum(ex.map(_oracle_interval, tasks))
        dt = time.perf_counter() - t0
    return dict(value=samples / dt, unit="vis/s", cores=workers,
                sample=f"{len(tasks)} intervals (the first {n_times} times x {int(term.n_gf)} channel intervals) "
                       f"solved to tol 1e-6 by the oracle in {workers} processes in {dt:.1f} s")


def leg_fp64(ctx, vis, term0, init_gains, int_bytes, stream, reps: int = 2):
    """The main workload's solve in FP64 (complex64 data widened on load, FP64
    products and sums), and the MIXED solution's difference from it: the
    largest over intervals of ||g_mixed - g_fp64||_2 / ||g_fp64||_2."""
    import numpy as np
    import torch
    mixed = term0.gains.clone()
    ms, st = [], None
    for _ in range(reps):
        term0.gains.copy_(init_gains)
        st = ctx.solve(vis, [term0], 0, tol=1e-6, max_iter=100, prec="fp64", stream=stream)
        ms.append(ctx.last_kernel_ms())
    it = st["iters"].cpu().numpy()
    g64 = term0.gains
    num = torch.linalg.vector_norm((mixed - g64).reshape(g64.shape[0], g64.shape[1], -1), dim=-1)
    den = torch.linalg.vector_norm(g64.reshape(g64.shape[0], g64.shape[1], -1), dim=-1)
    rel = float((num / den).max().item())
    term0.gains.copy_(mixed)
    gb = float(np.sum(np.maximum(it, 1) * int_bytes)) / 1e9
    k_ms = float(ms[-1])
    log(f"fp64: solve {k_ms:.1f} ms, mean iterations {it.mean():.2f} (max {it.max()}), {gb:.1f} GB -> "
        f"{gb / (k_ms * 1e-3):.0f} GB/s; MIXED against FP64: {rel:.2e}")
    return dict(kernel_ms=k_ms, mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                converged=float(st["converged"].float().mean().item()), algorithmic_gb=gb,
                achieved_gbs=gb / (k_ms * 1e-3), hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS,
                rel_err_mixed_vs_fp64=rel)


def cpu_baseline(prob, budget_s: float = 20.0):
    """The oracle as it stands, timed on host cores on a bounded sample of the
    same workload: whole intervals solved to tol 1e-6 until ~budget_s."""
    import numpy as np
    from oracle import solver as o_solver
    from synth.generate import slice_times, to_numpy_vis
    vis_h = to_numpy_vis(slice_times(prob.vis, 0, 1))
    term = prob.chain[0]
    one_t = term.copy(t_map=np.zeros(1, np.int32), n_gt=1, gains=term.gains[:1].copy(),
                      gain_flags=term.gain_flags[:1].copy())
    n_chan_int = int(np.sum(term.f_map == 0))
    done, samples, t0 = 0, 0, time.perf_counter()
    while done < one_t.n_gf:
        o_solver.solve_term(vis_h, [one_t], 0, tol=1e-6, max_iter=100, intervals=[(0, done)])
        done += 1
        samples += vis_h.data.shape[0] * n_chan_int
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=samples / dt, unit="vis/s", cores=1, kind="oracle",
                sample=f"{done} interval(s) of 1 time x {n_chan_int} channels x {vis_h.data.shape[0]} "
                       f"baselines solved to tol 1e-6 by the FP64 NumPy oracle in {dt:.1f} s")


def leg_tiny(ctx, dev, reps: int = 5):
    """The tiny configuration (7 antennas, 60 times x 16 channels, complex128, 24 intervals of
    10 times x 4 channels, sigma 0.01): the FP64 solve to tol 1e-6 on the GPU (median of reps,
    launch-latency bound) and the oracle on the whole problem on one core, with their
    largest per-interval relative difference."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from oracle import solver as o_solver
    from synth.generate import config_tiny, to_numpy_vis

    prob = config_tiny(sigma=0.01)
    vis_h = to_numpy_vis(prob.vis)
    vis_d = qc.device_vis(vis_h, dev)
    t0 = qc.device_term(prob.chain[0], dev)
    g0 = t0.gains.clone()
    stream = torch.cuda.current_stream()
    wall, kern = [], []
    for _ in range(reps + 1):
        t0.gains.copy_(g0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st = ctx.solve(vis_d, [t0], 0, tol=1e-6, max_iter=100, prec="fp64", stream=stream)
        torch.cuda.synchronize()
        wall.append(1e3 * (time.perf_counter() - ts))
        kern.append(ctx.last_kernel_ms())
    got = t0.gains.cpu().numpy()
    ts = time.perf_counter()
    ref, rst = o_solver.solve_term(vis_h, prob.chain, 0, tol=1e-6, max_iter=100)
    oracle_s = time.perf_counter() - ts
    w = ref[0].gains[..., [0, 3]]
    d = np.linalg.norm((got[..., [0, 3]] - w).reshape(w.shape[0], w.shape[1], -1), axis=-1)
    n = np.linalg.norm(w.reshape(w.shape[0], w.shape[1], -1), axis=-1)
    n_samples = int(vis_h.data.shape[0] * vis_h.data.shape[1])
    out = dict(samples=n_samples, intervals=int(t0.n_gt * t0.n_gf), gpu_wall_ms=float(np.median(wall[1:])),
               gpu_kernel_ms=float(np.median(kern[1:])), oracle_s=oracle_s, oracle_cores=1,
               vis_per_s_gpu=n_samples / (np.median(wall[1:]) * 1e-3), vis_per_s_oracle=n_samples / oracle_s,
               mean_iterations=float(st["iters"].float().mean().item()),
               iterations_equal=bool(np.array_equal(st["iters"].cpu().numpy(), rst["iters"])),
               rel_err_vs_oracle=float(np.max(d / n)))
    log(f"tiny: GPU {out['gpu_wall_ms']:.2f} ms (kernel {out['gpu_kernel_ms']:.3f} ms), oracle {oracle_s:.2f} s, "
        f"rel err {out['rel_err_vs_oracle']:.1e}")
    return out


def _oracle_fixed(task):
    """Oracle solve of one batch problem in fixed-iteration mode (pool worker)."""
    from oracle import solver as o_solver
    vis, term, k = task
    ref, _ = o_solver.solve_term(vis, [term], 0, tol=-1.0, max_iter=k)
    return ref[0].gains


def batch_oracle_stratified(probs, fp64_gains, dev, per_bucket: int = 6, n_pick: int = 32, k: int = 3,
                            workers: int = 0):
    """The oracle in fixed-iteration mode (k updates) on n_pick problems of the batch, stratified
    by the six size buckets of the batched launch (channel width <= 16 / <= 32 / wider x fewer or
    more than 65,536 samples per interval; the smallest problems of each bucket, for a bounded
    CPU time), in a pool of host processes, against the FP64 batched solve with the same k."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    from synth.generate import to_numpy_vis
    workers = workers or min(16, os.cpu_count() or 1)
    keyed = []
    for i, (vis, _, th) in enumerate(probs):
        n_ch = int(np.sum(np.asarray(th.f_map) == 0))
        rows = int(vis.data.shape[0]) // max(int(th.n_gt), 1)
        w = 0 if n_ch <= 16 else (1 if n_ch <= 32 else 2)
        z = 0 if rows * n_ch < (1 << 16) else 1
        keyed.append((w * 2 + z, int(vis.data.shape[0]) * int(vis.data.shape[1]), i))
    picked = []
    for b in range(6):
        cands = sorted(x for x in keyed if x[0] == b)
        picked += [x[2] for x in cands[:per_bucket]]
    rest = sorted((x for x in keyed if x[2] not in picked), key=lambda x: x[1])
    picked += [x[2] for x in rest[:max(0, n_pick - len(picked))]]
    picked = picked[:n_pick]
    tasks = [(to_numpy_vis(probs[i][0]), probs[i][2], k) for i in picked]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                             initializer=_one_blas_thread) as ex:
        refs = list(ex.map(_oracle_fixed, tasks))
    dt = time.perf_counter() - t0
    errs = []
    for i, ref in zip(picked, refs):
        g = fp64_gains[i].cpu().numpy()
        sel = [0, 3] if probs[i][2].kind == "diag" else [0, 1, 2, 3]
        a, w = g[..., sel], ref[..., sel]
        d = np.linalg.norm((a - w).reshape(w.shape[0], w.shape[1], -1), axis=-1)
        n = np.linalg.norm(w.reshape(w.shape[0], w.shape[1], -1), axis=-1)
        errs.append(float(np.max(d / np.maximum(n, 1e-300))))
    samples = int(sum(t[0].data.shape[0] * t[0].data.shape[1] for t in tasks))
    return dict(problems=picked, buckets=sorted(set(x[0] for x in keyed if x[2] in picked)), updates=k,
                samples=samples, oracle_s=dt, cores=workers, max_rel_err_fp64_vs_oracle=max(errs))


def leg_batch(ctx, dev, n_problems: int = 256, steps: int = 3):
    """Uneven batch: n_problems independent problems (antennas U{16..64}, times U{20..200},
    channels U{16..256}, dropped rows, diag / c2x2 50/50) solved to tol 1e-6 (MIXED) by
    (a) the plain loop of one qc_solve_interval per problem, (b) one graph launch of the
    batch with the default schedule, (c) the same after the autotuner.  Also FP64 vs MIXED
    on the GPU and both against the oracle on sampled problems."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from oracle import solver as o_solver
    from synth.generate import batch_shapes, config_batch_problem, to_numpy_vis

    t0 = time.perf_counter()
    shapes = batch_shapes(n_problems)
    probs = []
    for i, sh in enumerate(shapes):
        p = config_batch_problem(sh, i, device=dev)
        probs.append((p.vis, qc.device_term(p.chain[0], dev), p.chain[0]))
    torch.cuda.synchronize()
    n_samples = int(sum(int(v.data.shape[0]) * int(v.data.shape[1]) for v, _, _ in probs))
    log(f"batch: generated {n_problems} problems, {n_samples / 1e9:.3f}e9 samples in "
        f"{time.perf_counter() - t0:.1f} s; HBM in use {torch.cuda.memory_allocated() / 1e9:.1f} GB")
    init = [t.gains.clone() for _, t, _ in probs]
    stream = torch.cuda.current_stream()

    def reset():
        for (_, t, _), g0 in zip(probs, init):
            t.gains.copy_(g0)

    # (a) plain: one qc_solve_interval per problem, back to back
    reset()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    kern = 0.0
    for vis, t, _ in probs:
        ctx.solve(vis, [t], 0, tol=1e-6, max_iter=100, prec="mixed", stream=stream)
        kern += ctx.last_kernel_ms()
    torch.cuda.synchronize()
    plain_ms = 1e3 * (time.perf_counter() - tp)
    plain_gains = [t.gains.clone() for _, t, _ in probs]
    # (b) one graph launch, default schedule; (c) after tuning
    pairs = [(v, t) for v, t, _ in probs]
    b = qc.Batch(ctx, pairs, tol=1e-6, max_iter=100, prec="mixed", stream=stream)

    def timed_runs(k):
        ms = []
        for _ in range(k):
            reset()
            b.run(stream)
            ms.append(b.last_ms())
        return ms

    default_ms = timed_runs(steps)
    reset()                      # tune on the starting gains, as the timed runs solve
    tt = time.perf_counter()
    b.tune(reps=1)
    tune_s = time.perf_counter() - tt
    tuned_ms = timed_runs(steps)
    sched = b.schedule()
    iters = np.concatenate([st["iters"].cpu().numpy().ravel() for st in b.stats])
    alg_bytes = float(sum(np.sum(np.maximum(st["iters"].cpu().numpy().reshape(pass_bytes(v, th).shape), 1)
                                 * pass_bytes(v, th)) for st, (v, _, th) in zip(b.stats, probs)))
    mixed = [t.gains.clone() for _, t, _ in probs]
    d_plain = max(float((m - g).abs().max()) for m, g in zip(mixed, plain_gains))
    b.close()
    # FP64 on the GPU, same inputs
    bf = qc.Batch(ctx, pairs, tol=1e-6, max_iter=100, prec="fp64", stream=stream)
    reset()
    bf.run(stream)
    fp64_ms = bf.last_ms()
    fp64 = [t.gains.clone() for _, t, _ in probs]
    bf.close()
    # FP64 in fixed-iteration mode against the oracle on 32 problems stratified by bucket
    bk = qc.Batch(ctx, pairs, tol=-1.0, max_iter=3, prec="fp64", stream=stream)
    reset()
    bk.run(stream)
    torch.cuda.synchronize()
    fixed = [t.gains.clone() for _, t, _ in probs]
    bk.close()
    strat = batch_oracle_stratified(probs, fixed, dev)
    log(f"batch: oracle on {len(strat['problems'])} stratified problems ({strat['samples'] / 1e6:.1f}M samples, "
        f"{strat['updates']} updates) in {strat['oracle_s']:.1f} s on {strat['cores']} processes; FP64 batched "
        f"within {strat['max_rel_err_fp64_vs_oracle']:.1e}")

    def rel(a, w, kind):
        a, w = a.cpu().numpy(), np.asarray(w)
        if kind == "diag":
            a, w = a[..., [0, 3]], w[..., [0, 3]]
        nt, nf = w.shape[:2]
        d = np.linalg.norm((a - w).reshape(nt, nf, -1), axis=-1)
        n = np.linalg.norm(w.reshape(nt, nf, -1), axis=-1)
        return float(np.max(d / np.maximum(n, 1e-300)))

    e_mf = max(rel(m, f.cpu().numpy(), t0_.kind) for m, f, (_, _, t0_) in zip(mixed, fp64, probs))
    # oracle on the smallest problems of each term type (bounded CPU time)
    order = np.argsort([int(v.data.shape[0]) * int(v.data.shape[1]) for v, _, _ in probs])
    picked, seen = [], {"diag": 0, "c2x2": 0}
    for i in order:
        k = probs[i][2].kind
        if seen[k] < 2:
            picked.append(int(i))
            seen[k] += 1
    e_mo, e_fo = 0.0, 0.0
    for i in picked:
        vis, _, term_h = probs[i]
        ref, _ = o_solver.solve_term(to_numpy_vis(vis), [term_h], 0, tol=1e-6, max_iter=100)
        e_mo = max(e_mo, rel(mixed[i], ref[0].gains, term_h.kind))
        e_fo = max(e_fo, rel(fp64[i], ref[0].gains, term_h.kind))
    out = dict(problems=n_problems, samples=n_samples,
               plain_wall_ms=plain_ms, plain_kernel_ms=kern,
               batch_default_ms=float(np.mean(default_ms)), batch_tuned_ms=float(np.mean(tuned_ms)),
               tune_s=tune_s, batch_fp64_ms=fp64_ms,
               vis_per_s_plain=n_samples / (plain_ms * 1e-3),
               vis_per_s_batched=n_samples / (np.mean(tuned_ms) * 1e-3),
               speedup_vs_plain=plain_ms / float(np.mean(tuned_ms)),
               mean_iterations=float(iters.mean()), schedule=sched,
               algorithmic_gb=alg_bytes / 1e9,
               achieved_gbs_batched=alg_bytes / (np.mean(tuned_ms) * 1e-3) / 1e9,
               hbm_frac_batched=alg_bytes / (np.mean(tuned_ms) * 1e-3) / 1e9 / HBM_PEAK_GBS,
               max_abs_diff_batched_vs_plain=d_plain,
               rel_err_mixed_vs_fp64_gpu=e_mf, rel_err_mixed_vs_oracle=e_mo, rel_err_fp64_vs_oracle=e_fo,
               oracle_problems=picked, oracle_stratified_fixed_iterations=strat)
    log(f"batch: plain {plain_ms:.1f} ms (kernels {kern:.1f}), graph default {np.mean(default_ms):.1f} ms, "
        f"tuned {np.mean(tuned_ms):.1f} ms (tuning {tune_s:.1f} s), fp64 {fp64_ms:.1f} ms; "
        f"mixed vs fp64 {e_mf:.2e}, vs oracle {e_mo:.2e}")
    return out


def leg_warm(ctx, dev, n_sets: int = 5, n_time_train: int = 625, epochs: int = 30):
    """Learned warm start: a 2-layer MLP (hidden 256) trained by the library's own kernels on
    n_sets x n_time_train x 16 solver-labelled MeerKAT-like intervals (64 antennas, 1 time x 64
    channels, random diagonal gains); evaluated on held-out data of the full 600 x 1024 shape
    against the unit-gain start: iterations to tol 1e-6 and wall time including the feature
    pass, the inference and the solver's unit-gain fallback."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc, warmstart
    from synth.generate import config_meerkat

    t0 = time.perf_counter()
    feats, labels, info = warmstart.training_set(ctx, n_sets=n_sets, n_time=n_time_train, device=dev, log=log)
    gen_s = time.perf_counter() - t0
    net = warmstart.WarmStartNet(ctx, n_ant=64, n_hid=256, device=dev, seed=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = net.train(feats, labels, epochs=epochs, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    n_train = int(feats.shape[0])
    del feats, labels
    torch.cuda.empty_cache()
    held = config_meerkat(device=dev, n_time=600, kind="diag", gain_mode="random", cfg_id=50, seed_block=0)
    n_samples = int(held.vis.data.shape[0]) * int(held.vis.data.shape[1])
    stream = torch.cuda.current_stream()
    res = {}
    for mode in ("unit", "warm", "unit", "warm"):          # second round timed warm
        t = qc.device_term(held.chain[0], dev)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        if mode == "unit":
            st = ctx.solve(held.vis, [t], 0, tol=1e-6, max_iter=100, prec="mixed", stream=stream)
        else:
            st = warmstart.solve_with_warm_start(ctx, net, held.vis, t, stream=stream)
        torch.cuda.synchronize()
        res[mode] = dict(ms=1e3 * (time.perf_counter() - ts), iters=float(st["iters"].float().mean().item()),
                         restarted=float(st["restarted"].float().mean().item()),
                         converged=float(st["converged"].float().mean().item()), gains=t.gains)
    lb = learned_batched(ctx, net, dev)
    om = oracle_mlp_step(net)
    # agreement of the two solutions (model-level, gauge free): max |g_p conj(g_q)| difference
    gu, gw = res["unit"]["gains"], res["warm"]["gains"]
    pu = gu[:, :, :, 0, 0, None] * gu[:, :, None, :, 0, 0].conj()
    pw = gw[:, :, :, 0, 0, None] * gw[:, :, None, :, 0, 0].conj()
    agree = float(((pu - pw).abs().max() / pu.abs().max()).item())
    out = dict(train_intervals=n_train, train_set_s=gen_s, train_s=train_s, epochs=epochs,
               loss_first=hist[0], loss_last=hist[-1], label_mean_iterations=info["mean_iterations"],
               held_out_samples=n_samples,
               unit_iters=res["unit"]["iters"], warm_iters=res["warm"]["iters"],
               iterations_saved=res["unit"]["iters"] - res["warm"]["iters"],
               unit_ms=res["unit"]["ms"], warm_ms=res["warm"]["ms"],
               time_saved_frac=1.0 - res["warm"]["ms"] / res["unit"]["ms"],
               restarted_frac=res["warm"]["restarted"], converged_frac=res["warm"]["converged"],
               model_agreement=agree, params=net.n_params, learned_batched=lb,
               gpu_train_step_ms=1e3 * train_s / max(1, epochs * (n_train // 256)), oracle_mlp_step=om)
    log(f"warm start: {n_train} training intervals ({gen_s:.1f} s to make), training {train_s:.1f} s, "
        f"loss {hist[0]:.4f} -> {hist[-1]:.4f}; held-out iterations unit {out['unit_iters']:.2f} "
        f"warm {out['warm_iters']:.2f}; time unit {out['unit_ms']:.1f} ms warm {out['warm_ms']:.1f} ms")
    return out


def oracle_mlp_step(net, batch: int = 256, reps: int = 5):
    """The oracle's FP64 training step of the same network (forward, MSE gradient, backward,
    Adam) on one host core, batch 256, from the trained parameters: the median of reps."""
    import numpy as np
    from oracle import warmstart as o_ws
    rng = np.random.default_rng(7)
    params = net.params.double().cpu().numpy()
    I, H, O = net.n_in, net.n_hid, net.n_out
    x = rng.standard_normal((batch, I))
    tgt = rng.standard_normal((batch, O))
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    times = []
    for k in range(reps):
        t0 = time.perf_counter()
        y, pre = o_ws.forward(params, x, I, H, O)
        _, dy = o_ws.mse(y, tgt)
        g = o_ws.backward(params, x, pre, dy, I, H, O)
        params, m, v = o_ws.adam(params, g, m, v, 1e-3, 0.9, 0.999, 1e-8, k + 1)
        times.append(time.perf_counter() - t0)
    return dict(ms=1e3 * float(np.median(times)), batch=batch, cores=1)


def learned_batched(ctx, net, dev, n_problems: int = 32, reps: int = 2):
    """Learned + batched against plain, at tol 1e-6 (MIXED): n_problems held-out problems of
    uneven size (64 antennas, times U{8..40}, 256 / 512 / 1024 channels, whole rows dropped at a
    fraction U(0, 0.3), 10% sample flags, random diagonal gains, intervals 1 time x 64 channels)
    solved four ways, each timed on the wall clock from the first launch to the last result:
    plain (one qc_solve_interval per problem from unit gains), batched (one graph launch from
    unit gains), learned (per problem: feature pass, MLP, gain write, solve with the unit-gain
    fallback) and learned + batched (the batch's feature pass over every interval, the MLP
    over all of them, the batch's gain write, then one graph launch with per-problem fallback
    references).  The two batched paths run on their autotuned schedules, as the batch leg's
    tuned graph (the tuning itself is not timed; the warm batch is tuned from its learned
    start); their default schedules are timed too."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc, warmstart
    from synth.generate import config_meerkat

    g = np.random.default_rng(np.random.SeedSequence([2412, 51]))
    made = []
    t0 = time.perf_counter()
    for i in range(n_problems):
        n_time = int(g.integers(8, 41))
        n_chan = int(g.choice([256, 512, 1024]))
        drop = float(g.uniform(0.0, 0.3))
        p = config_meerkat(device=dev, n_time=n_time, n_chan=n_chan, f_int=64, kind="diag", gain_mode="random",
                           cfg_id=51, seed_block=i, row_drop=drop)
        made.append((p.vis, qc.device_term(p.chain[0], dev)))
    # chi^2 at unit gains of every interval in one array, problem after problem
    # (the batch's row order), each problem's fallback reference a slice of it
    ref_all = torch.empty(sum(int(t.n_gt) * int(t.n_gf) for _, t in made), dtype=torch.float64, device=dev)
    probs, o = [], 0
    for v, t in made:
        n_i = int(t.n_gt) * int(t.n_gf)
        probs.append((v, t, ref_all[o:o + n_i], t.gains.clone()))
        o += n_i
    torch.cuda.synchronize()
    n_samples = int(sum(int(v.data.shape[0]) * int(v.data.shape[1]) for v, _, _, _ in probs))
    n_int = int(sum(int(t.n_gt) * int(t.n_gf) for _, t, _, _ in probs))
    log(f"learned+batched: {n_problems} problems, {n_int} intervals, {n_samples / 1e9:.3f}e9 samples "
        f"({time.perf_counter() - t0:.1f} s to make)")
    stream = torch.cuda.current_stream()

    def reset():
        for _, t, _, g0 in probs:
            t.gains.copy_(g0)

    b_unit = qc.Batch(ctx, [(v, t) for v, t, _, _ in probs], tol=1e-6, max_iter=100, prec="mixed", stream=stream)
    b_warm = qc.Batch(ctx, [(v, t, r) for v, t, r, _ in probs], tol=1e-6, max_iter=100, prec="mixed",
                      stream=stream)

    def run(mode):
        stats = None
        if mode == "tune":
            reset()
            b_unit.tune()
            reset()
            net.init_gains_batch(b_warm, ref_all, stream=stream)
            b_warm.tune()
            return None
        if mode == "plain":
            stats = [ctx.solve(v, [t], 0, tol=1e-6, max_iter=100, prec="mixed", stream=stream)
                     for v, t, _, _ in probs]
        elif mode.startswith("batched"):
            b_unit.run(stream)
            stats = b_unit.stats
        elif mode == "learned":
            stats = []
            for v, t, r, _ in probs:
                net.init_gains(v, t, stream=stream, chisq_out=r)
                stats.append(ctx.solve(v, [t], 0, tol=1e-6, max_iter=100, prec="mixed", stream=stream,
                                       chisq_ref=r.reshape(int(t.n_gt), int(t.n_gf))))
        else:
            net.init_gains_batch(b_warm, ref_all, stream=stream)
            b_warm.run(stream)
            stats = b_warm.stats
        return stats

    out = {}
    t_tune = 0.0
    for mode in ("plain", "batched_default", "learned_batched_default", "tune", "batched", "learned",
                 "learned_batched"):
        if mode == "tune":
            ts = time.perf_counter()
            run(mode)
            torch.cuda.synchronize()
            t_tune = time.perf_counter() - ts
            continue
        best = None
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            stats = run(mode)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - ts)
            best = ms if best is None else min(best, ms)
        it = np.concatenate([s["iters"].cpu().numpy().ravel() for s in stats])
        rs = np.concatenate([s["restarted"].cpu().numpy().ravel() for s in stats])
        cv = np.concatenate([s["converged"].cpu().numpy().ravel() for s in stats])
        out[mode] = dict(ms=best, vis_per_s=n_samples / (best * 1e-3), mean_iterations=float(it.mean()),
                         restarted_frac=float(rs.mean()), converged_frac=float(cv.mean()))
    b_unit.close()
    b_warm.close()
    res = dict(problems=n_problems, intervals=n_int, samples=n_samples, **out, tune_s=t_tune,
               speedup_learned_batched_vs_plain=out["plain"]["ms"] / out["learned_batched"]["ms"],
               speedup_batched_vs_plain=out["plain"]["ms"] / out["batched"]["ms"],
               speedup_learned_vs_plain=out["plain"]["ms"] / out["learned"]["ms"],
               speedup_learned_batched_default_vs_plain=out["plain"]["ms"] / out["learned_batched_default"]["ms"])
    log("learned+batched: " + ", ".join(f"{m} {out[m]['ms']:.1f} ms ({out[m]['mean_iterations']:.2f} updates)"
                                       for m in out) +
        f"; learned+batched vs plain {res['speedup_learned_batched_vs_plain']:.2f}x")
    del probs
    torch.cuda.empty_cache()
    return res


def leg_chain(ctx, dev, n_epoch: int = 2):
    """Jones chain + directions: 64 antennas, 300 times x 512 channels, 4 clusters of 5
    sources (one model direction each); chain K (delay, 60 times x band) . B (bandpass,
    all times x 1 channel) . G (gain, 1 time x band) . dE (direction-dependent, 16 times x
    128 channels); Fourier-peak delay start, then n_epoch epochs over the chain to tol 1e-6
    (MIXED), then the residual."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from synth.generate import config_chain

    t0 = time.perf_counter()
    p = config_chain(device=dev)
    torch.cuda.synchronize()
    vis = p.vis
    n_samples = int(vis.data.shape[0]) * int(vis.data.shape[1])
    log(f"chain: generated {n_samples / 1e9:.3f}e9 samples x {vis.model.shape[2]} directions in "
        f"{time.perf_counter() - t0:.1f} s")
    chain = [qc.device_term(t, dev) for t in p.chain]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ctx.delay_init(vis, chain[0], ref_ant=0, stream=stream)
    torch.cuda.synchronize()
    t_delay = time.perf_counter() - ts
    k_start = chain[0].params.clone()
    log(f"chain: delay initial estimate {1e3 * t_delay:.1f} ms")
    terms = []
    for e in range(n_epoch):
        for n, t in enumerate(chain):
            t1 = time.perf_counter()
            st = ctx.solve(vis, chain, n, tol=1e-6, max_iter=100, prec="mixed", stream=stream)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t1)
            it = st["iters"].cpu().numpy()
            gb = float(np.sum(np.maximum(it, 1) * pass_bytes(vis, p.chain[n]))) / 1e9
            terms.append(dict(epoch=e, term=t.name, intervals=int(t.n_gt * t.n_gf),
                              split_parts=int(ctx.last_split_parts()), ms=ms,
                              mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                              converged=float(st["converged"].float().mean().item()),
                              algorithmic_gb=gb, achieved_gbs=gb / (ms * 1e-3)))
            d = terms[-1]
            log(f"chain: epoch {e} term {d['term']}: {d['ms']:.0f} ms, {d['intervals']} intervals, "
                f"parts {d['split_parts']}, mean iterations {d['mean_iterations']:.2f} (max "
                f"{d['max_iterations']}), converged {100 * d['converged']:.1f}%, {gb:.1f} GB -> "
                f"{d['achieved_gbs']:.0f} GB/s")
    t2 = time.perf_counter()
    resid = ctx.residual(vis, chain, stream=stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    t_total = t_end - ts
    use = (vis.flag == 0)
    rms = float(torch.sqrt((resid.abs() ** 2).sum(-1)[use].mean() / 4).item())
    sigma = float(p.meta["sigma"])
    out = dict(samples=n_samples, directions=int(vis.model.shape[2]), delay_init_ms=1e3 * t_delay,
               terms=terms, residual_ms=1e3 * (t_end - t2), total_s=t_total,
               vis_per_s=n_samples / t_total, residual_rms=rms, noise_rms=sigma * math.sqrt(2),
               bytes_per_sample_pass=float(np.mean(pass_bytes(vis, p.chain[0]))) / max(
                   float(np.mean(interval_samples(vis, p.chain[0]))), 1.0))
    log(f"chain: delay init {1e3 * t_delay:.1f} ms; " + "; ".join(
        f"{d['term']}{d['epoch']} {d['ms']:.0f} ms it {d['mean_iterations']:.1f} parts {d['split_parts']}"
        for d in terms) + f"; total {t_total:.2f} s; residual rms {rms:.4f} (noise {sigma * math.sqrt(2):.4f})")
    del resid
    try:
        out["oracle_k_pass"] = oracle_k_pass(p, chain)
    except Exception as e:   # report, keep the leg
        out["oracle_k_pass"] = {"error": f"{type(e).__name__}: {e}"}
    out["predicted_model"] = chain_predicted(ctx, p, k_start, n_epoch, stream)
    out["de_levenberg_marquardt"] = chain_de_lm(ctx, p, k_start, n_epoch, stream)
    return out


def oracle_k_pass(p, chain_d, n_times: int = 60, n_chan: int = 4):
    """The oracle's rate on the delay term's blocks (one accumulation pass of K, chain at the
    solved gains, 4 directions) over a slice of one K interval: its first 60 times x the first
    4 channels, on one host core (the full interval of 60 times x 512 channels would need tens
    of GB of host memory for the oracle's per-sample 4x4 blocks)."""
    import numpy as np
    from paper_2412_10072_amd import qc
    from oracle import solver as o_solver
    from synth.generate import slice_times, to_numpy_vis

    vis_h = to_numpy_vis(slice_times(p.vis, 0, n_times))
    vis_k = vis_h.copy(data=np.ascontiguousarray(vis_h.data[:, :n_chan]),
                       model=np.ascontiguousarray(vis_h.model[:, :n_chan]),
                       weight=np.ascontiguousarray(vis_h.weight[:, :n_chan]),
                       flag=np.ascontiguousarray(vis_h.flag[:, :n_chan]), chan_freq=vis_h.chan_freq[:n_chan])
    chain_h = []
    for t in chain_d:
        h = qc.host_term(t)
        chain_h.append(h.copy(t_map=np.asarray(h.t_map)[:n_times], f_map=np.asarray(h.f_map)[:n_chan]))
    rows = np.arange(vis_k.data.shape[0])
    s = o_solver.samples_of(vis_k, rows, np.arange(n_chan))
    t0 = time.perf_counter()
    o_solver.accumulate(vis_k, chain_h, 0, s)
    dt = time.perf_counter() - t0
    n = int(rows.size * n_chan)
    log(f"chain: oracle K pass over {n / 1e6:.2f}M samples in {dt:.1f} s ({n / dt:.3g} samples/s, 1 core)")
    return dict(samples=n, seconds=dt, samples_per_s=n / dt, cores=1,
                sample=f"first {n_times} times x first {n_chan} channels of one K interval, one pass")


def chain_de_lm(ctx, p, k_start, n_epoch, stream):
    """The same chain solve with the direction-dependent term dE under Levenberg-Marquardt
    damping instead of the half steps its default (AUTO) takes, from the same delay start:
    dE's updates and time per epoch, and the residual."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc

    vis = p.vis
    dev = vis.data.device
    chain = [qc.device_term(t, dev) for t in p.chain]
    chain[0].params.copy_(k_start)
    terms = []
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for e in range(n_epoch):
        for n, t in enumerate(chain):
            damping = "lm" if t.name == "dE" else "auto"
            t1 = time.perf_counter()
            st = ctx.solve(vis, chain, n, tol=1e-6, max_iter=100, prec="mixed", damping=damping, stream=stream)
            torch.cuda.synchronize()
            it = st["iters"].cpu().numpy()
            terms.append(dict(epoch=e, term=t.name, damping=damping, ms=1e3 * (time.perf_counter() - t1),
                              mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                              converged=float(st["converged"].float().mean().item()),
                              split_parts=int(ctx.last_split_parts())))
    resid = ctx.residual(vis, chain, stream=stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    use = (vis.flag == 0)
    rms = float(torch.sqrt((resid.abs() ** 2).sum(-1)[use].mean() / 4).item())
    out = dict(terms=terms, total_s=t_end - ts, residual_rms=rms)
    log("chain, dE under LM: " + "; ".join(
        f"{d['term']}{d['epoch']} {d['ms']:.0f} ms it {d['mean_iterations']:.1f}" for d in terms) +
        f"; total {t_end - ts:.2f} s; residual rms {rms:.4f}")
    return out


def chain_predicted(ctx, p, k_start, n_epoch, stream):
    """The same chain solve with the model predicted inside every pass from the 20 point
    components (qc_solve_interval_sky / qc_residual_sky) instead of read: per sample and
    pass 32 B data + 16 B weights + 1 B flag (+ 24 B of baseline coordinates per row) against
    the 177 B with the stored 4-direction model; from the same delay start."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc

    vis = p.vis
    dev = vis.data.device
    lm, fl, dr = [], [], []
    for d, (l, m, flux) in enumerate(p.meta["sky"]):
        lm.append(torch.stack([torch.as_tensor(l, dtype=torch.float64, device=dev).reshape(-1),
                               torch.as_tensor(m, dtype=torch.float64, device=dev).reshape(-1)], -1))
        fl.append(torch.as_tensor(flux, dtype=torch.float64, device=dev).reshape(-1))
        dr.append(torch.full((fl[-1].numel(),), d, dtype=torch.int32, device=dev))
    lm, fl, dr = torch.cat(lm).contiguous(), torch.cat(fl), torch.cat(dr).contiguous()
    n_comp = int(fl.numel())
    stokes = torch.zeros(n_comp, 4, dtype=torch.float64, device=dev)
    stokes[:, 0] = fl
    sky = qc.Sky(lm=lm, stokes=stokes, spi=torch.zeros(n_comp, dtype=torch.float64, device=dev),
                 ref_freq=torch.full((n_comp,), 1.4e9, dtype=torch.float64, device=dev), comp_dir=dr,
                 uvw=p.meta["uvw"].to(torch.float64).contiguous(), n_dir=len(p.meta["sky"]))
    vis_s = vis.copy(model=None)
    chain = [qc.device_term(t, dev) for t in p.chain]
    chain[0].params.copy_(k_start)
    n_samples = int(vis.data.shape[0]) * int(vis.data.shape[1])
    n_rows = int(vis.data.shape[0])
    per_sample = 32 + 4 * int(vis.weight.shape[2]) + 1
    terms = []
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for e in range(n_epoch):
        for n, t in enumerate(chain):
            t1 = time.perf_counter()
            st = ctx.solve_sky(vis_s, sky, chain, n, tol=1e-6, max_iter=100, prec="mixed", stream=stream)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t1)
            it = st["iters"].cpu().numpy()
            n_int = int(t.n_gt * t.n_gf)
            gb = float(np.maximum(it, 1).mean()) * (n_samples * per_sample + n_rows * 24 * int(t.n_gf)) / 1e9
            terms.append(dict(epoch=e, term=t.name, split_parts=int(ctx.last_split_parts()), ms=ms,
                              mean_iterations=float(it.mean()),
                              converged=float(st["converged"].float().mean().item()), algorithmic_gb=gb))
    t2 = time.perf_counter()
    resid = ctx.residual_sky(vis_s, sky, chain, stream=stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    use = (vis.flag == 0)
    rms = float(torch.sqrt((resid.abs() ** 2).sum(-1)[use].mean() / 4).item())
    out = dict(components=n_comp, bytes_per_sample_pass=per_sample, terms=terms, residual_ms=1e3 * (t_end - t2),
               total_s=t_end - ts, vis_per_s=n_samples / (t_end - ts), residual_rms=rms)
    log("chain, predicted model: " + "; ".join(
        f"{d['term']}{d['epoch']} {d['ms']:.0f} ms it {d['mean_iterations']:.1f}" for d in terms) +
        f"; residual {1e3 * (t_end - t2):.1f} ms; total {t_end - ts:.2f} s; residual rms {rms:.4f}")
    return out


def leg_params(ctx, dev):
    """Phase-only and amplitude-only solves (real parameters, one per hand) on the
    MeerKAT shape: 64 antennas, 600 times x 1024 channels, complex64, interval
    1 time x 64 channels, truth phases (unit amplitude) or amplitudes (zero
    phase), MIXED to tol 1e-6; then a delay-and-offset solve (phase offset and
    delay per hand) with interval 1 time x 1024 channels from the delay
    initial estimate."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from synth.generate import config_meerkat

    out = {}
    for kind in ("phase", "amplitude"):
        p = config_meerkat(device=dev, kind=kind)
        torch.cuda.synchronize()
        term = qc.device_term(p.chain[0], dev)
        init = term.params.clone()
        ms, st = [], None
        for rep in range(3):
            term.params.copy_(init)
            st = ctx.solve(p.vis, [term], 0, tol=1e-6, max_iter=100, prec="mixed")
            ms.append(ctx.last_kernel_ms())
        it = st["iters"].cpu().numpy()
        gb = float(np.sum(np.maximum(it, 1) * pass_bytes(p.vis, p.chain[0]))) / 1e9
        k_ms = float(np.mean(ms[1:]))
        out[kind] = dict(kernel_ms=k_ms, mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                         converged=float(st["converged"].float().mean().item()), algorithmic_gb=gb,
                         achieved_gbs=gb / (k_ms * 1e-3), hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS)
        log(f"params: {kind}-only solve {k_ms:.1f} ms, mean iterations {it.mean():.2f} (max {it.max()}), "
            f"{gb:.1f} GB -> {gb / (k_ms * 1e-3):.0f} GB/s")
        del p, term, init
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    # delay and phase offset per hand (the K term), interval 1 time x the band, from the
    # Fourier-peak delay start; too few intervals to fill the chip, so split across it
    p = config_meerkat(device=dev, kind="delay_offset", f_int=1024)
    torch.cuda.synchronize()
    term = qc.device_term(p.chain[0], dev)
    ts = time.perf_counter()
    ctx.delay_init(p.vis, term, ref_ant=0)
    ctx.sync()
    t_init = 1e3 * (time.perf_counter() - ts)
    init = term.params.clone()
    ms, st = [], None
    for rep in range(3):
        term.params.copy_(init)
        st = ctx.solve(p.vis, [term], 0, tol=1e-6, max_iter=100, prec="mixed")
        ms.append(ctx.last_kernel_ms())
    parts = ctx.last_split_parts()
    it = st["iters"].cpu().numpy()
    gb = float(np.sum(np.maximum(it, 1) * pass_bytes(p.vis, p.chain[0]))) / 1e9
    k_ms = float(np.mean(ms[1:]))
    host = qc.host_term(term)
    rel = host.params - host.params[:, :, :1]          # referenced to antenna 0: the data fix differences
    d_tau = rel[..., [1, 3]] - p.truth[0].params[..., [1, 3]]
    out["delay_offset"] = dict(kernel_ms=k_ms, delay_init_ms=t_init, split_parts=int(parts),
                               mean_iterations=float(it.mean()), max_iterations=int(it.max()),
                               converged=float(st["converged"].float().mean().item()), algorithmic_gb=gb,
                               achieved_gbs=gb / (k_ms * 1e-3), hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS,
                               max_delay_error_ps=float(1e12 * np.abs(d_tau).max()))
    log(f"params: delay_offset solve {k_ms:.1f} ms in {parts} parts (delay init {t_init:.1f} ms), mean "
        f"iterations {it.mean():.2f} (max {it.max()}), {gb:.1f} GB -> {gb / (k_ms * 1e-3):.0f} GB/s, "
        f"max delay error {1e12 * np.abs(d_tau).max():.2f} ps")
    del p, term, init
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def leg_pointing(ctx, dev, reps: int = 3):
    """Pointing offsets through the primary beam (one parameter pair per antenna whose
    effect differs by direction): the chain workload's array, band and 4 clustered model
    directions (64 antennas, 300 times x 512 channels, complex64), one pointing term with
    intervals of 30 times x the band, MIXED to tol 1e-6 from zero offsets."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from synth.generate import config_pointing
    p = config_pointing(device=dev)
    torch.cuda.synchronize()
    term = qc.device_term(p.chain[0], dev)
    init = term.params.clone()
    ms, st = [], None
    for rep in range(reps):
        term.params.copy_(init)
        st = ctx.solve(p.vis, [term], 0, tol=1e-6, max_iter=100, prec="mixed")
        ms.append(ctx.last_kernel_ms())
    parts = ctx.last_split_parts()
    it = st["iters"].cpu().numpy()
    gb = float(np.sum(np.maximum(it, 1) * pass_bytes(p.vis, p.chain[0]))) / 1e9
    k_ms = float(np.mean(ms[1:]))
    err = float(np.abs(qc.host_term(term).params - p.truth[0].params).max() / p.meta["fwhm"])
    n_samples = int(p.vis.data.shape[0]) * int(p.vis.data.shape[1])
    out = dict(samples=n_samples, directions=int(p.vis.model.shape[2]), intervals=int(it.size), parts=int(parts),
               solve_ms=k_ms, mean_iterations=float(it.mean()), max_iterations=int(it.max()),
               converged=float(st["converged"].float().mean().item()), algorithmic_gb=gb,
               achieved_gbs=gb / (k_ms * 1e-3), hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS,
               sample_passes_per_s=float(np.sum(np.maximum(it, 1)) * n_samples / it.size) / (k_ms * 1e-3),
               max_offset_error_beamwidths=err)
    log(f"pointing: {it.size} intervals x {parts} parts, solve {k_ms:.1f} ms, mean iterations {it.mean():.2f} "
        f"(max {it.max()}), {gb:.1f} GB -> {gb / (k_ms * 1e-3):.0f} GB/s, largest offset error {err:.2e} "
        f"beam widths")
    del p, term, init
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def flag_pass_bytes(vis) -> dict:
    """Algorithmic HBM bytes per sample of qc_mad_flag's passes: the statistic
    pass reads the residual (4 complex), the weights and the flag and writes
    the statistic; each radix-select histogram pass reads the statistic (11-bit
    digits: 3 passes per selection in FP32, 6 in FP64; two selections, median
    and MAD); the apply pass reads the statistic and the flag and writes the
    output flag.  one_pass is the floor of any method: read the residual,
    weights and flag once, write the flag."""
    import torch
    c64 = vis.data.dtype == torch.complex64
    e = 4 if c64 else 8
    wcorr = int(vis.weight.shape[-1])
    stat = 8 * e + wcorr * e + 1 + e
    hist = 2 * (3 if c64 else 6) * e
    apply = e + 1 + 1
    return dict(stat=stat, hist=hist, apply=apply, total=stat + hist + apply,
                one_pass=8 * e + wcorr * e + 1 + 1)


LANE_SLOTS_PER_S = 256 * 64 * 2.4e9       # CUs x lanes issued per cycle x clock
PREDICT_SLOTS = 16                          # minimal issue slots per component-sample (flat, unpolarised)


def leg_predict(ctx, prob, reps: int = 3):
    """DFT prediction of the main workload's model (MeerKAT shape, 20 point
    sources) from its component list, then the plain solve from that model;
    and the same components with full Stokes and spectral indices."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    vis = prob.vis
    dev = vis.data.device
    n_row, n_chan = int(vis.data.shape[0]), int(vis.data.shape[1])
    l, m, flux = prob.meta["sky"][0]
    n_comp = int(l.shape[0])
    uvw = prob.meta["uvw"]
    lm = torch.stack([l, m], 1).contiguous()
    st = torch.zeros(n_comp, 4, dtype=torch.float64, device=dev)
    st[:, 0] = flux
    spi = torch.zeros(n_comp, dtype=torch.float64, device=dev)
    nu0 = torch.full((n_comp,), 1.284e9, dtype=torch.float64, device=dev)
    d = torch.zeros(n_comp, dtype=torch.int32, device=dev)
    model = torch.empty_like(vis.model)
    evals = n_row * n_chan * n_comp
    peak = LANE_SLOTS_PER_S / PREDICT_SLOTS
    out = dict(samples=n_row * n_chan, components=n_comp, comp_samples=evals, peak_comp_samples_per_s=peak)

    def timed(stk, sp):
        ms = []
        for _ in range(reps):
            ctx.predict(uvw, vis.chan_freq, lm, stk, sp, nu0, d, n_dir=1, dtype="c64", out=model)
            ms.append(ctx.last_kernel_ms())
        return float(np.mean(ms[1:]))

    k_ms = timed(st, spi)
    rate = evals / (k_ms * 1e-3)
    out["flat_unpolarised"] = dict(kernel_ms=k_ms, comp_samples_per_s=rate, alu_frac=rate / peak,
                                   write_gbs=32.0 * n_row * n_chan / (k_ms * 1e-3) / 1e9)
    log(f"predict: {n_comp} components x {n_row * n_chan / 1e9:.3f}e9 samples in {k_ms:.1f} ms -> "
        f"{rate:.3e} component-samples/s ({100 * rate / peak:.1f}% of the ALU bound)")
    # the solve from the predicted model (the same iterations as from the generator's model)
    term = qc.device_term(prob.chain[0], dev)
    stt = ctx.solve(vis.copy(model=model), [term], 0, tol=1e-6, max_iter=100, prec="mixed")
    s_ms = ctx.last_kernel_ms()
    it = stt["iters"].cpu().numpy()
    out["solve_from_predicted"] = dict(kernel_ms=s_ms, mean_iterations=float(it.mean()),
                                       converged=float(stt["converged"].float().mean().item()))
    log(f"predict: solve from the predicted model {s_ms:.1f} ms, mean iterations {it.mean():.2f}")
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    stp = st.clone()
    stp[:, 1:] = 0.05 * flux[:, None] * (2 * torch.rand(n_comp, 3, generator=g, device=dev, dtype=torch.float64) - 1)
    spp = -0.7 + 0.2 * torch.rand(n_comp, generator=g, device=dev, dtype=torch.float64)
    k2 = timed(stp, spp)
    out["full_stokes_spectral"] = dict(kernel_ms=k2, comp_samples_per_s=evals / (k2 * 1e-3))
    log(f"predict: full Stokes with spectral indices {k2:.1f} ms")
    del model
    return out


def leg_robust(ctx, vis, resid, chain, nu: float = 2.0, reps: int = 3):
    """Robust weights from the main solve's residual and the weights of the
    corrected data through the solved gains (MeerKAT shape, complex64).
    Algorithmic bytes per sample: robust weights 2 x (32 residual + 16
    weights + 1 flag) + 16 written = 114; corrected weights 16 read + 16
    written = 32 (gains and row metadata are negligible)."""
    import numpy as np
    import torch
    n = int(vis.data.shape[0]) * int(vis.data.shape[1])
    w = torch.empty_like(vis.weight)
    out = {}
    for name, fn, bps in (("robust_weights", lambda: ctx.robust_weights(vis, resid, nu=nu, out=w, want_s2=False), 114),
                          ("corrected_weights", lambda: ctx.corrected_weights(vis, chain, out=w), 32)):
        ms = []
        for _ in range(reps):
            fn()
            ms.append(ctx.last_kernel_ms())
        k_ms = float(np.mean(ms[1:]))
        gb = bps * n / 1e9
        out[name] = dict(kernel_ms=k_ms, bytes_per_sample=bps, algorithmic_gb=gb, achieved_gbs=gb / (k_ms * 1e-3),
                         hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS)
        log(f"robust: {name} {k_ms:.1f} ms, {gb:.1f} GB -> {gb / (k_ms * 1e-3):.0f} GB/s")
    del w
    return out


def leg_interp(ctx, term, n_time: int, n_chan: int, reps: int = 3):
    """The main solve's gains (one solution per time and 64 channels)
    interpolated to one per time and channel (1GC-style transfer onto a finer
    grid): FP64 amplitude and short-arc phase per Jones entry."""
    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    dev = term.gains.device
    t_src = torch.arange(term.n_gt, dtype=torch.float64, device=dev) * 8.0
    f_src = 856e6 + (torch.arange(term.n_gf, dtype=torch.float64, device=dev) + 0.5) * 64 * (856e6 / n_chan)
    f_dst = torch.linspace(856e6, 1712e6, n_chan, dtype=torch.float64, device=dev)
    dst = term.copy()
    dst.n_gf = n_chan
    dst.f_map = torch.arange(n_chan, dtype=torch.int32, device=dev)
    dst.gains = torch.empty(term.n_gt, n_chan, *term.gains.shape[2:], dtype=torch.complex128, device=dev)
    dst.gain_flags = torch.zeros(term.n_gt, n_chan, *term.gains.shape[2:4], dtype=torch.int8, device=dev)
    ms = []
    for _ in range(reps):
        ctx.interp_term(term, t_src, f_src, dst, t_src, f_dst, int(term.gains.shape[2]))
        ms.append(ctx.last_kernel_ms())
    k_ms = float(np.mean(ms[1:]))
    n_out = int(dst.gains.numel() // 4)
    out = dict(points_out=n_out, kernel_ms=k_ms, points_per_s=n_out / (k_ms * 1e-3),
               written_gb=dst.gains.numel() * 16 / 1e9)
    log(f"interp: {term.n_gt} x {term.n_gf} -> {term.n_gt} x {n_chan} solutions ({n_out / 1e6:.1f}M antenna points) "
        f"in {k_ms:.2f} ms")
    del dst
    return out


def leg_flag(ctx, vis, resid, k: float = 5.0, reps: int = 3):
    """MAD outlier flagging of the main solve's residual (MeerKAT shape,
    1.24e9 samples), over all samples at once and per baseline."""
    import numpy as np
    import torch
    n_samples = int(vis.data.shape[0]) * int(vis.data.shape[1])
    pb = flag_pass_bytes(vis)
    out = dict(samples=n_samples, k=k, bytes_per_sample=pb)
    flags = torch.empty_like(vis.flag)
    n_in = int((vis.flag != 0).sum().item())
    for mode in ("global", "baseline"):
        ms, wall = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, n_new, st = ctx.mad_flag(vis, resid, mode=mode, k=k, flag_out=flags, stats=True)
            wall.append(1e3 * (time.perf_counter() - t0))
            ms.append(ctx.last_kernel_ms())
        k_ms = float(np.mean(ms[1:]))
        gb = pb["total"] * n_samples / 1e9
        stn = st.cpu().numpy()
        out[mode] = dict(kernel_ms=k_ms, wall_ms=float(np.mean(wall[1:])), new_flags=int(n_new),
                         new_flag_frac=n_new / max(n_samples - n_in, 1), algorithmic_gb=gb,
                         achieved_gbs=gb / (k_ms * 1e-3), hbm_frac=gb / (k_ms * 1e-3) / HBM_PEAK_GBS,
                         one_pass_ms_at_peak=pb["one_pass"] * n_samples / 1e9 / HBM_PEAK_GBS * 1e3,
                         median=float(np.median(stn[:, 0])), mad=float(np.median(stn[:, 1])))
        log(f"flag {mode}: {k_ms:.1f} ms kernels ({np.mean(wall[1:]):.1f} ms wall), {n_new} new flags "
            f"({100 * n_new / max(n_samples - n_in, 1):.3f}%), {gb:.1f} GB -> {gb / (k_ms * 1e-3):.0f} GB/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-time", type=int, default=600)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="tiny,fp64,flag,robust,interp,predict,batch,warm,chain,params,pointing",
                    help="comma list of extra legs: tiny, fp64, flag, robust, interp, predict, batch, warm, chain, "
                         "params, pointing (or none)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy a 4 GiB device buffer once (a kernel of known traffic for HBM counters)")
    ap.add_argument("--traffic-record", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "ALG_BYTES"),
                    help="write the solve kernel's traffic record from two rocprofv3 csv runs and exit")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(args.traffic_record[0], args.traffic_record[1], float(args.traffic_record[2]))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver shards by solution intervals with no communication, "
              "and this implementation runs on a single MI355X; --gpus above 1 is not supported.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2412_10072_amd import qc
    from synth.generate import config_meerkat

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(1 << 32, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 4294967296 B read + 4294967296 B written")
        del src, dst
        torch.cuda.empty_cache()
    t0 = time.perf_counter()
    prob = config_meerkat(device=dev, n_time=args.n_time)
    torch.cuda.synchronize()
    vis = prob.vis
    n_row, n_chan = int(vis.data.shape[0]), int(vis.data.shape[1])
    n_samples = n_row * n_chan
    log(f"generated {n_row} rows x {n_chan} channels ({n_samples / 1e9:.3f}e9 samples) in "
        f"{time.perf_counter() - t0:.1f} s; HBM in use {torch.cuda.memory_allocated() / 1e9:.1f} GB")

    ctx = qc.Context(0)
    term0 = qc.device_term(prob.chain[0], dev)
    init_gains = term0.gains.clone()
    chain = [term0]
    resid = torch.empty_like(vis.data)
    stream = torch.cuda.current_stream()
    n_int = int(term0.n_gt * term0.n_gf)
    int_bytes = pass_bytes(vis, prob.chain[0])
    int_samples = interval_samples(vis, prob.chain[0])

    def step():
        term0.gains.copy_(init_gains)
        st = ctx.solve(vis, chain, 0, tol=1e-6, max_iter=100, prec="mixed", damping="auto", stream=stream)
        ms = ctx.last_kernel_ms()
        ctx.residual(vis, chain, out=resid, stream=stream)
        return st, ms

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.sync()
    kern_ms, alg_bytes, iters_all = [], [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        st, ms = step()
        kern_ms.append(ms)
        it = st["iters"].cpu().numpy()
        iters_all.append(it)
        alg_bytes.append(float(np.sum(np.maximum(it, 1) * int_bytes)))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ctx.sync()

    ms_per_step = 1e3 * t_total / args.steps
    value = n_samples / (t_total / args.steps)
    copy_gbs = copy_bandwidth(dev)
    k_ms = float(np.mean(kern_ms))
    achieved = float(np.mean(alg_bytes)) / (k_ms * 1e-3) / 1e9
    it = iters_all[-1]
    conv = float(st["converged"].float().mean().item())
    log(f"step {ms_per_step:.1f} ms; solve kernel {k_ms:.1f} ms; iterations mean {it.mean():.2f} "
        f"min {it.min()} max {it.max()}; converged {conv * 100:.1f}%; "
        f"algorithmic {np.mean(alg_bytes) / 1e9:.1f} GB per solve -> {achieved:.0f} GB/s")

    out = {
        "metric": "calibrated visibilities/s at 1e-6 tol, %HBM peak; learned+batched vs plain",
        "value": value,
        "unit": "vis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"MeerKAT-shaped full-Jones solve: 64 antennas, {args.n_time} times x 1024 "
                               "channels, complex64, 20 sources, 10% flags, interval 1 time x 64 channels, "
                               "tol 1e-6, plain MIXED solver + residual pass",
                   "samples": n_samples, "intervals": n_int, "mean_iterations": float(it.mean()),
                   "iterations_histogram": {int(k): int(v) for k, v in zip(*np.unique(it, return_counts=True))},
                   "converged_fraction": conv},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_solve_fused",
                     "kernel_ms": k_ms, "algorithmic_gb_per_launch": float(np.mean(alg_bytes)) / 1e9,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "flop_per_sample_pass": FLOP_PER_SAMPLE_C2X2,
                     "fp32_tflops": FLOP_PER_SAMPLE_C2X2 * float(np.sum(np.maximum(it, 1) * int_samples))
                                    / (k_ms * 1e-3) / 1e12},
    }
    tr = measured_traffic()
    if tr is not None and args.n_time == 600:
        out["roofline"]["traffic"] = tr["traffic_bytes"] / 1e9
        out["roofline"]["traffic_unit"] = "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
        try:
            out["cpu_baseline"]["all_cores"] = cpu_baseline_pool(prob, n_times=16)
            log(f"cpu baseline: 1 core {out['cpu_baseline']['value']:.3g} vis/s, "
                f"{out['cpu_baseline']['all_cores']['cores']} processes "
                f"{out['cpu_baseline']['all_cores']['value']:.3g} vis/s")
        except Exception as e:   # report, keep the main measurement
            out["cpu_baseline"]["all_cores"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"all-core oracle baseline failed: {e}")
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    if legs:
        out["legs"] = {}
    if "tiny" in legs:
        try:
            out["legs"]["tiny"] = leg_tiny(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["tiny"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"tiny leg failed: {e}")
    if "fp64" in legs:
        try:
            out["legs"]["fp64"] = leg_fp64(ctx, vis, term0, init_gains, int_bytes, stream)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["fp64"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"fp64 leg failed: {e}")
    if "flag" in legs:
        try:
            out["legs"]["flag"] = leg_flag(ctx, vis, resid)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["flag"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"flag leg failed: {e}")
    if "robust" in legs:
        try:
            out["legs"]["robust"] = leg_robust(ctx, vis, resid, chain)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["robust"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"robust leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "interp" in legs:
        try:
            out["legs"]["interp"] = leg_interp(ctx, term0, args.n_time, n_chan)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["interp"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"interp leg failed: {e}")
    if "predict" in legs:
        try:
            out["legs"]["predict"] = leg_predict(ctx, prob)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["predict"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"predict leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if legs:
        del prob, vis, resid, chain, term0, init_gains
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "batch" in legs:
        try:
            out["legs"]["batch"] = leg_batch(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["batch"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"batch leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "warm" in legs:
        try:
            out["legs"]["warm"] = leg_warm(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["warm"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"warm leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "params" in legs:
        try:
            out["legs"]["params"] = leg_params(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["params"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"params leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "pointing" in legs:
        try:
            out["legs"]["pointing"] = leg_pointing(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["pointing"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"pointing leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if "chain" in legs:
        try:
            out["legs"]["chain"] = leg_chain(ctx, dev)
        except Exception as e:   # report, keep the main measurement
            out["legs"]["chain"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"chain leg failed: {e}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
