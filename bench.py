#!/usr/bin/env python3
"""Throughput of distributed FastMNMF on one MI355X, as one JSON line.

A step is one whole job on one synthetic mixture already resident in HBM:
reset the state to its initial values, run the workload's iterations
(IP sweep + eqs. (8), (9), (10) each), evaluate the cost (13) and separate the
sources with the per-subarray Wiener filter.  The reported value is
iterations per second over the timed steps (whole job, one GPU); the
iterations are replayed from HIP graphs (``--no-graph``: plain launches).

Workload (default ``paper_4x4``): F=513 bins, T=625 frames, four subarrays of
four mics (M=16), N=5 sources, K=16 bases, 100 iterations, complex64 with the
IP solves in FP64.  Inputs are seeded synthetic mixtures (see
``paper_2605_19388_amd/synth.py``).

Extra objects on the line:
* ``roofline`` -- the slower of the two kernels with the largest share of an
  iteration: its algorithmic HBM bytes per launch divided by its average
  duration, measured with HIP events around each of its launches over a pass
  of the same steps right after the timed region (``kernels`` lists both);
  ``iteration`` prices the whole iteration (28 B per F*T*M bin) at the
  measured time per iteration;
* ``cpu_baseline`` -- the FP64 NumPy oracle timed on this host on a bounded
  sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FastMNMF iterations/sec (F·T·M bins/s) at 4×4 mics N=5; % MFMA/HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # dense FP64 (vector and matrix cores) of MI355X

# Algorithmic HBM bytes per F*T*M bin for each streaming kernel of the FP32 path
# (complex64 X = 8 B, FP32 P = 4 B).  One iteration's schedule reads X twice and
# writes P once and reads it twice: 28 B per bin.  Shape-specialised kernels map onto the
# same steps (k_gramd_f / k_gram_f: covariances; k_pw_f: powers and the W coefficients;
# k_h_f: the H coefficients; k_g_f: the g update).
BYTES_PER_BIN = {"k_gram": 8.0, "k_gramd": 8.0, "k_pw": 12.0, "k_h": 4.0, "k_g": 4.0}
ITER_BYTES_PER_BIN = 28.0  # the whole iteration: 2 x 8 (X) + 3 x 4 (P written once, read twice)
KERNEL_SOURCE = os.path.join(ROOT, "paper_2605_19388_amd", "csrc", "dfm_fast.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_paper_4x4.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper_4x4")
    ap.add_argument("--iters", type=int, default=None, help="iterations per step (default: the workload's)")
    ap.add_argument("--cpu-sample-iters", type=int, default=4)
    ap.add_argument("--cpu-sample-iters-1t", type=int, default=2,
                    help="iterations of the single-thread oracle leg")
    ap.add_argument("--gram-bf16", action="store_true",
                    help="covariances of eq. (14) from BF16 operands on the matrix cores (FP32 sums)")
    ap.add_argument("--batch", type=int, default=0, metavar="B",
                    help="B uneven mixtures (2-8 subarrays of 4 mics, N in {3, 5, 8}, T in [200, 2000], F=513, "
                         "K=16, complex64), tiles from the autotuner, stepped as one batch of graph replays and "
                         "one after another; prints its own JSON line")
    ap.add_argument("--grad", type=int, default=0, metavar="N",
                    help="time the gradient of the cost after N unrolled MM iterations (forward with "
                         "checkpoints + hand-written reverse pass) and print its own JSON line")
    ap.add_argument("--grad-full", action="store_true",
                    help="with --grad: unroll full iterations (eq. (14), the IP sweep, then the MM updates) "
                         "instead of MM iterations with Q fixed")
    ap.add_argument("--no-graph", action="store_true",
                    help="plain kernel launches instead of HIP graph replays (for comparison)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the oracle's NumPy/BLAS pools (default: as the host sets them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    ap.add_argument("--mixtures", type=int, default=1,
                    help="B > 1: per-kernel durations with the Infinity Cache cold, from B copies of the "
                         "mixture stepped round-robin one iteration at a time (prints its own JSON line)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-mb run into the traffic file and exit (no GPU needed)")
    return ap.parse_args()


def source_digest():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def pmc_summary(fetch_csv, write_csv, copy_mb):
    """Per-kernel HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for the calibration copy of copy_mb MiB."""
    import csv
    import collections

    def per_kernel(path):
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            vals[name].append(float(r["Counter_Value"]))
        return vals

    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = per_kernel(path)
        copies = [v for k, vs in vals.items() if "copyBuffer" in k for v in vs]
        if not copies:
            raise SystemExit(f"{path}: no calibration copy found (run the profiled bench with --copy-mb)")
        measured = max(copies)  # KiB the counter reports for the copy of copy_mb MiB
        factor = copy_mb * 1024.0 / measured
        out[counter] = {"calibration_kib": measured, "expected_kib": copy_mb * 1024.0, "factor": factor,
                        "kernels": {short_name(k): statistics_mean(vs) * factor * 1024.0
                                    for k, vs in vals.items() if k.startswith("void dfm::")}}
    return out


def statistics_mean(v):
    return sum(v) / len(v)


def short_name(symbol):
    """'void dfm::fast::k_pw_f<float, 5, 16, 4, 4>(...)' -> 'k_pw_f'."""
    return symbol.split("(")[0].replace("void ", "").split("<")[0].split("::")[-1]


def load_traffic(kernel):
    """Measured HBM bytes per launch of `kernel` from the committed counter summary, or None
    if there is none or the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def cpu_baseline(w, X64, W0, H0, n_iter, threads=0):
    """Time the FP64 oracle, unmodified, on n_iter iterations of the same full-size workload
    (with its thread pools limited to `threads` if that is positive)."""
    import contextlib

    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import dfmnmf as D

    Q, g = w["Q"], w["g"]
    with threadpool_limits(limits=threads) if threads > 0 else contextlib.nullcontext():
        st = D.iterate(X64, Q, g, W0, H0, w["mics"], 1)          # warm-up
        t0 = time.perf_counter()
        D.iterate(X64, *st, w["mics"], n_iter)
        dt = time.perf_counter() - t0
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    return {"value": n_iter / dt, "unit": "iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_iter} of {w['iters']} iterations of {w['name']} at full size "
                      f"(F={w['F']}, T={w['T']}, M={w['M']}, N={w['N']}, K={w['K']}) after 1 warm-up "
                      f"iteration, NumPy FP64, {dt:.1f} s",
            "ms_per_iteration": 1e3 * dt / n_iter, "bins_per_s": n_iter * w["F"] * w["T"] * w["M"] / dt,
            "cpu": _cpu_model(), "np_version": np.__version__}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cold_mixtures(args):
    """Kernel durations with the 256 MB Infinity Cache cold.

    One mixture's working set (X 41 MB, P 20.5 MB, planes, lambda: about 80 MB at paper_4x4)
    stays cache-resident from kernel to kernel, so the default run measures cache-assisted
    bandwidth.  Here B plans, each with its own device copy of the mixture, are stepped
    round-robin one iteration at a time: between two uses of one plan's data the other B - 1
    plans move (B - 1) x ~150 MB, so with B = 8 every launch reads and writes HBM.  Each kernel
    is timed with events around its own launches on every plan.  step(1) also refreshes
    lambda once per call (one extra kernel per iteration, included in `iterations_per_s`).
    """
    import numpy as np
    import torch

    from paper_2605_19388_amd import DistributedFastMNMF, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B, rounds = args.mixtures, max(args.steps, 2) * 4
    w = synth.make(args.workload)
    F, T, M, N, K, mics = w["F"], w["T"], w["M"], w["N"], w["K"], w["mics"]
    X32 = w["X"].astype(np.complex64)
    dev = torch.device("cuda:0")
    plans = [DistributedFastMNMF(X32, mics, N, K, W=w["W"].astype(np.float32), H=w["H"].astype(np.float32),
                                 Q=w["Q"].astype(np.complex64), g=w["g"].astype(np.float32), device=dev)
             for _ in range(B)]
    names = plans[0].kernel_names()
    plans[0].step(2)
    warm = plans[0].kernel_times(reps=args.kernel_reps)
    log(f"[bench] {B} copies of {w['name']}; warm per-kernel us: " +
        ", ".join(f"{k}={v * 1e3:.1f}" for k, v in warm.items()))

    def rounds_of(n):
        for _ in range(n):
            for p in plans:
                p.step(1)

    rounds_of(2)
    torch.cuda.synchronize()
    cold = {}
    for k in names:
        for p in plans:
            p.profile_kernel(k, max_launches=rounds + 4)
        rounds_of(rounds)
        torch.cuda.synchronize()
        tot, n = 0.0, 0
        for p in plans:
            ms, cnt = p.profile_read()
            p.profile_kernel(None)
            tot += ms * cnt
            n += cnt
        cold[k] = tot / max(n, 1)
        log(f"[bench] {k}: cold {cold[k] * 1e3:.2f} us (warm {warm[k] * 1e3:.2f}) over {n} launches")
    t0 = time.perf_counter()
    rounds_of(rounds)
    torch.cuda.synchronize()
    ips = rounds * B / (time.perf_counter() - t0)
    for p in plans:
        p.sync_status()
    bins = F * T * M
    roof = {}
    for k, ms in cold.items():
        base = k[:-2] if k.endswith("_f") else k
        if base in BYTES_PER_BIN:
            gbs = BYTES_PER_BIN[base] * bins / (ms * 1e-3) / 1e9
            roof[k] = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out = {"mode": "cold_mixtures", "workload": w["name"], "mixtures": B, "rounds": rounds,
           "iterations_per_s": round(ips, 1),
           "per_kernel_us_cold": {k: round(v * 1e3, 2) for k, v in cold.items()},
           "per_kernel_us_warm": {k: round(v * 1e3, 2) for k, v in warm.items()},
           "iteration_us_cold": round(sum(cold.values()) * 1e3, 2),
           "iteration_us_warm": round(sum(warm.values()) * 1e3, 2),
           "roofline_cold": roof}
    print(json.dumps(out), flush=True)


def _live_kernel_times(p, one_step, steps, iters, kernels):
    """Average duration (ms) of each kernel in `kernels` over `steps` whole steps, measured with
    a pair of HIP events recorded on the launch stream around each of its launches (one kernel
    per pass; while a kernel is profiled the launches are plain, since events cannot bracket one
    kernel inside a graph replay)."""
    import torch
    out = {}
    for k in kernels:
        p.profile_kernel(k, max_launches=iters * steps + 8)
        for _ in range(steps):
            one_step()
        torch.cuda.synchronize()
        ms, n = p.profile_read()
        p.profile_kernel(None)
        out[k] = (ms, n)
    return out


def grad_timing(args):
    """Whole-job time of the unrolled-iteration gradient on the workload: reset, N MM (or, with
    --grad-full, full) iterations with per-iteration checkpoints, the cost, the reverse pass (FP64
    internally)."""
    import numpy as np
    import torch

    from paper_2605_19388_amd import DistributedFastMNMF, synth

    w = synth.make(args.workload)
    F, T, M, N, K, mics = w["F"], w["T"], w["M"], w["N"], w["K"], w["mics"]
    dev = torch.device("cuda:0")
    p = DistributedFastMNMF(w["X"].astype(np.complex64), mics, N, K, W=w["W"].astype(np.float32),
                            H=w["H"].astype(np.float32), Q=w["Q"].astype(np.complex64), g=w["g"].astype(np.float32),
                            device=dev)
    init = {k: getattr(p, k).clone() for k in ("Q", "g", "W", "H")}

    def one():
        for k, v in init.items():
            getattr(p, k).copy_(v)
        tape = p.iter_forward(args.grad) if args.grad_full else p.mm_forward(args.grad)
        cost = p.nll()
        return cost, (p.iter_backward(tape) if args.grad_full else p.mm_backward(tape))

    for _ in range(max(args.warmup, 1)):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"mode": "grad", "workload": w["name"], "map": "full iterations" if args.grad_full else "mm iterations",
                      "iterations": args.grad, "ms_per_gradient": round(1e3 * dt, 3),
                      "gradients_per_s": round(1.0 / dt, 2), "dtype": "f32 state, f64 reverse pass"}), flush=True)


def batch_timing(args):
    """Batched against one-after-another stepping of B uneven mixtures (the same plans, tiles from
    the autotuner), `--iters` iterations (default 100) per step."""
    import numpy as np
    import torch

    from paper_2605_19388_amd import autotune, binding, synth

    B, iters = args.batch, args.iters or 100
    rng = np.random.Generator(np.random.PCG64(1000))
    shapes = [(513, int(rng.integers(200, 2001)), (4,) * int(rng.integers(2, 9)), int(rng.choice([3, 5, 8])), 16)
              for _ in range(B)]
    # Tiles per shape class, tuned on a 65-bin excerpt of each class (the tile sets the frames per
    # workgroup of the per-frame kernels, which depends on T, N and M, not on F).
    t0 = time.perf_counter()
    tiles = {}
    for F, T, mics, N, K in shapes:
        key = autotune.shape_key(F, T, mics, N, K)
        if key not in tiles:
            tiles[key], _ = autotune.tune(65, T, mics, N, K, iters=2, reps=1)
            if len(tiles) % 8 == 0:
                log(f"[bench] {len(tiles)} shape classes tuned")
    log(f"[bench] {len(tiles)} shape classes tuned in {time.perf_counter() - t0:.1f} s")
    plans = []
    for b, (F, T, mics, N, K) in enumerate(shapes):
        if b % 8 == 0:
            log(f"[bench] drawing mixture {b} of {B}")
        X = synth.mixture(F, T, mics, N, K, 1000 + b, mixing="delay").astype(np.complex64)
        Q, g, W, H = synth.initial_state(F, T, mics, N, K, 2000 + b)
        plans.append(binding.DistributedFastMNMF(X, mics, N, K, W=W.astype(np.float32), H=H.astype(np.float32),
                                                 Q=Q.astype(np.complex64), g=g.astype(np.float32),
                                                 tile=tiles[autotune.shape_key(F, T, mics, N, K)]))
        del X
    fast = sum(1 for p in plans if p.kernel_names()[0].endswith("_f"))
    log(f"[bench] {B} mixtures ({fast} on the specialised kernels), {iters} iterations per step")
    init = [{k: getattr(p, k).clone() for k in ("Q", "g", "W", "H")} for p in plans]

    def reset():
        for p, st in zip(plans, init):
            for k, v in st.items():
                getattr(p, k).copy_(v)

    batch = binding.Batch(plans)
    reset()
    batch.step(2)
    for p in plans:
        p.step(2)
    torch.cuda.synchronize()
    res = {}
    for mode in ("batched", "one_after_another"):
        ts = []
        for _ in range(max(args.steps, 1)):
            reset()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if mode == "batched":
                batch.step(iters)
            else:
                for p in plans:
                    p.step(iters)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        res[mode] = min(ts)
    bins = sum(F * T * sum(m) for F, T, m, _, _ in shapes)
    for p in plans:
        p.sync_status()
    out = {"mode": "batch", "mixtures": B, "specialised": fast, "iterations": iters,
           "shape_classes": len(tiles),
           "batched_s": round(res["batched"], 4), "one_after_another_s": round(res["one_after_another"], 4),
           "speedup": round(res["one_after_another"] / res["batched"], 3),
           "mixture_iterations_per_s": round(B * iters / res["batched"], 1),
           "bins_per_s": round(bins * iters / res["batched"], 1)}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.batch > 0:
        batch_timing(args)
        return
    if args.mixtures > 1:
        cold_mixtures(args)
        return
    if args.grad > 0:
        grad_timing(args)
        return
    if args.pmc_summary:
        copy_mb = args.copy_mb or 256
        t = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], copy_mb)
        kernels = sorted(set(t["FETCH_SIZE"]["kernels"]) | set(t["WRITE_SIZE"]["kernels"]))
        doc = {"workload": "paper_4x4", "source_sha256": source_digest(), "copy_mb": copy_mb,
               "calibration": {c: {k: v for k, v in t[c].items() if k != "kernels"} for c in t},
               "kernels": {k: {"fetch_bytes": t["FETCH_SIZE"]["kernels"].get(k, 0.0),
                               "write_bytes": t["WRITE_SIZE"]["kernels"].get(k, 0.0)} for k in kernels}}
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(doc, fh, indent=1)
        print(json.dumps(doc, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method is sharded across GPUs only by running independent mixtures).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_19388_amd import DistributedFastMNMF, binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.make(args.workload)
    iters = args.iters or w["iters"]
    F, T, M, N, K, mics = w["F"], w["T"], w["M"], w["N"], w["K"], w["mics"]
    X32 = w["X"].astype(np.complex64)
    W32, H32 = w["W"].astype(np.float32), w["H"].astype(np.float32)
    dev = torch.device("cuda:0")
    flags = (binding.F_NO_GRAPH if args.no_graph else 0) | (binding.F_GRAM_BF16 if args.gram_bf16 else 0)
    p = DistributedFastMNMF(X32, mics, N, K, W=W32, H=H32, Q=w["Q"].astype(np.complex64),
                            g=w["g"].astype(np.float32), device=dev, flags=flags)
    init = {k: getattr(p, k).clone() for k in ("Q", "g", "W", "H")}
    S = torch.empty((N, F, T, M), dtype=torch.complex64, device=dev)

    def reset():
        for k, v in init.items():
            getattr(p, k).copy_(v)

    def one_step():
        reset()
        p.step(iters)
        nll = p.nll()
        p.separate(out=S)
        return nll

    log(f"[bench] workload {w['name']} F={F} T={T} mics={mics} N={N} K={K} iters/step={iters} "
        f"launches={'plain' if args.no_graph else 'graph replays'}")
    if args.copy_mb:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.copy_mb} MiB done")
    # Per-kernel durations back to back (outside the timed region) to rank the kernels.
    reset()
    p.step(2)
    ktimes = p.kernel_times(reps=args.kernel_reps)
    reset()
    log("[bench] per-kernel average (back to back): " + ", ".join(f"{k}={v * 1e3:.1f}us" for k, v in ktimes.items()))
    top = sorted(ktimes, key=ktimes.get, reverse=True)[:2]

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # Timed region: whole steps, nothing else on the stream.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    nll = None
    for _ in range(args.steps):
        nll = one_step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    value = iters * args.steps / elapsed
    bins = F * T * M
    log(f"[bench] {args.steps} steps in {elapsed:.4f} s (events {gpu_ms:.2f} ms); nll={nll:.6e}")
    # The same steps again with each of the two slowest kernels bracketed by HIP events.
    live = _live_kernel_times(p, one_step, args.steps, iters, top)
    p.sync_status()
    for k, (ms, n) in live.items():
        log(f"[bench] {k}: {ms * 1e3:.2f} us avg over {n} launches (events on the launch stream)")
    dominant = max(live, key=lambda k: live[k][0])

    def kernel_roof(k):
        ms, n = live[k]
        base = k[:-2] if k.endswith("_f") else k   # shape-specialised variants
        traffic = load_traffic(k) if w["name"] == "paper_4x4" else None  # counters taken on paper_4x4
        if base not in BYTES_PER_BIN:
            return {"kernel": k, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": None, "traffic": traffic, "avg_us": round(ms * 1e3, 3), "launches": n}
        alg = BYTES_PER_BIN[base] * bins
        gbs = alg / (ms * 1e-3) / 1e9
        return {"kernel": k, "bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_us": round(ms * 1e3, 3),
                "launches": n, "algorithmic_bytes_per_launch": alg}

    roof = kernel_roof(dominant)
    roof["kernels"] = [kernel_roof(k) for k in top]
    # Whole iteration: the reference schedule's bytes over the measured time per iteration (the
    # per-step reset, cost and separation included, so this is a lower bound).
    it_bytes = ITER_BYTES_PER_BIN * bins
    it_us = 1e6 * elapsed / (args.steps * iters)
    roof["iteration"] = {"bytes": it_bytes, "us": round(it_us, 3),
                         "achieved": round(it_bytes / (it_us * 1e-6) / 1e9, 2), "unit": "GB/s",
                         "frac": round(it_bytes / (it_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                         "kernel_sum_us": round(sum(ktimes.values()) * 1e3, 2)}

    # The contraction of eq. (14) runs on the FP64 matrix cores (16x16x4) when a subarray has
    # more than four mics.  Priced at the flops the kernel executes (16 x 16 tiles of
    # (1/y)[mu] times the M_l^2 packed products, K = 4 frames: 2 M_l^3 per frame and subarray)
    # and, for reference, at eq. (14) as written (a complex multiply-add is 8 flops: 8 M_l^3).
    gram_mfma = None
    if "k_gram_f" in ktimes and max(mics) > 4:
        executed = 2.0 * sum(ml ** 3 for ml in mics) * F * T
        written = 8.0 * sum(ml ** 3 for ml in mics) * F * T
        sec = ktimes["k_gram_f"] * 1e-3
        gram_mfma = {"bound": "mfma", "kernel": "k_gram_f", "achieved": round(executed / sec / 1e12, 2),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(executed / sec / 1e12 / FP64_PEAK_TFLOPS, 4),
                     "flops_executed_per_launch": executed, "flops_as_written_per_launch": written,
                     "as_written_tflops": round(written / sec / 1e12, 2),
                     "avg_us": round(ktimes["k_gram_f"] * 1e3, 2)}
    out = {"metric": METRIC, "value": round(value, 3), "unit": "iterations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": w["name"], "F": F, "T": T, "mics": list(mics), "N": N, "K": K,
                      "iterations_per_step": iters, "bins_per_iteration": bins,
                      "launches": "plain" if args.no_graph else "graph replays",
                      "covariances": "bf16 operands, fp32 sums" if args.gram_bf16 else "fp32 operands, fp64 sums",
                      "step": "reset + iterations + cost (13) + Wiener separation"},
           "bins_per_s": round(value * bins, 1),
           "per_kernel_us": {k: round(v * 1e3, 2) for k, v in ktimes.items()},
           "roofline": roof}
    if gram_mfma:
        out["roofline_gram"] = gram_mfma
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (all threads, then one) ...")
        X64, W64, H64 = X32.astype(np.complex128), W32.astype(np.float64), H32.astype(np.float64)
        cb = cpu_baseline(w, X64, W64, H64, args.cpu_sample_iters, args.cpu_threads)
        cb["single_thread"] = cpu_baseline(w, X64, W64, H64, args.cpu_sample_iters_1t, 1)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
