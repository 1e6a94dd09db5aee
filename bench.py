#!/usr/bin/env python3
"""Benchmark of the batched FP32 C2C FFT on one MI355X.

Headline workload: forward FFT, N = 2048, batch 32768 (2^26 complex64
elements: 512 MiB read + 512 MiB written per step), inputs resident in HBM.
One step = one fft_execute of that batch.  Also measured in the same run:
the forward + adjoint pair of the differentiable FFT (N = 2048, batch
16384), the per-N sweep (every N = 2..2048 at 2^26 elements, forward and
inverse), a plain 512 MiB copy kernel as the practical bandwidth ceiling,
and the FP64 CPU oracle on a bounded sample (cpu_baseline).

Prints ONE JSON line.  Times come from HIP events recorded on the stream
the kernels are launched on (torch's current stream).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "FP32 C2C FFT GFLOP/s (5NlogN) & HBM GB/s at N=2048; fwd+adjoint vs plain fwd"
KERNEL_SOURCES = ["paper_2203_09384_amd/csrc/device_fft.hpp", "paper_2203_09384_amd/csrc/fft_c32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fft_c32_n2048_b32768.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_launches(fn, steps, warmup, torch):
    """Average ms per call of fn() over `steps` back-to-back calls on the
    current stream, bracketed by HIP events; also min/median of per-call
    events for the distribution."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    total = e0.elapsed_time(e1)
    return total / steps


def per_call_distribution(fn, reps, torch):
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return {"min_ms": ts[0], "median_ms": ts[len(ts) // 2], "mean_ms": sum(ts) / len(ts)}


def cpu_baseline(n, budget_s=12.0):
    """FP64 oracle on a bounded sample of the headline workload."""
    import numpy as np
    import oracle
    from paper_2203_09384_amd import synth
    threads = oracle.default_threads()
    probe = synth.uniform_complex(synth.SEED_PLAIN, (threads * 4, n), key=(n, 1234)).astype(np.complex128)
    t0 = time.perf_counter()
    oracle.forward(probe, threads=threads)
    dt = time.perf_counter() - t0
    per = dt / probe.shape[0]
    count = int(max(threads * 4, min(1 << 15, budget_s / max(per, 1e-9))))
    x = synth.uniform_complex(synth.SEED_PLAIN, (count, n), key=(n, 4321)).astype(np.complex128)
    t0 = time.perf_counter()
    oracle.forward(x, threads=threads)
    dt = time.perf_counter() - t0
    flops = 5.0 * n * math.log2(n) * count
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} forward transforms of N={n} (FP64 recursive radix-2, {dt:.1f} s)",
            "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline kernel (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the batched transforms are independent, so the path "
              f"has no multi-GPU step to run here (got --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_09384_amd import api, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    props = torch.cuda.get_device_properties(0)
    log(f"[bench] device {props.name} {getattr(props, 'gcnArchName', '')} CUs={props.multi_processor_count}")

    # ---------------------------------------------------------------- headline
    n = 2048
    total = 1 << 26
    batch = total // n
    log("[bench] generating 2^26 seeded complex64 inputs")
    x_np = synth.uniform_complex(synth.SEED_PLAIN, (total,), key=(0,))
    x_all = torch.from_numpy(x_np).to(dev)
    del x_np
    y_all = torch.empty_like(x_all)
    x = x_all.view(batch, n)
    y = y_all.view(batch, n)
    plan = api.Plan(n, batch, -1)
    desc = plan.describe()
    log(f"[bench] headline plan {desc}")
    ms = time_launches(lambda: plan.execute(x, y), args.steps, args.warmup, torch)
    bytes_alg = 16.0 * total
    gbps = bytes_alg / (ms * 1e-3) / 1e9
    gflops = 5.0 * n * math.log2(n) * batch / (ms * 1e-3) / 1e9
    log(f"[bench] headline fwd N=2048: {ms * 1e3:.1f} us, {gbps:.0f} GB/s, {gflops:.0f} GFLOP/s")
    out = {
        "metric": METRIC, "value": round(gflops, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FP32 C2C forward FFT, N=2048, batch 32768 (2^26 complex64, "
                               "512 MiB in + 512 MiB out), out of place, re/im uniform[-1,1) seeded",
                   "n": n, "batch": batch, "ept": desc["ept"], "wg": desc["wg"],
                   "radices": desc["radices"], "seed": synth.SEED_PLAIN},
    }
    traffic = None
    khash = kernel_hash()
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == khash:
            traffic = tr.get("bytes_per_launch")
    out["roofline"] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic,
                       "kernel": "k_fft_c32<11,4,256,-1>", "kernel_hash": khash,
                       "algorithmic_bytes_per_launch": bytes_alg}
    out["headline_distribution"] = per_call_distribution(lambda: plan.execute(x, y), 50, torch)
    out["gflops_fwd_2048"] = round(gflops, 1)
    out["gbps_fwd_2048"] = round(gbps, 1)

    if not args.only_headline:
        # ------------------------------------------------------------ copy ceiling
        ms_copy = time_launches(lambda: torch.mul(x_all, 1.0, out=y_all), args.steps, args.warmup, torch)
        out["copy_ceiling_GBps"] = round(bytes_alg / (ms_copy * 1e-3) / 1e9, 1)
        log(f"[bench] copy 512 MiB: {out['copy_ceiling_GBps']} GB/s")

        # ------------------------------------------------------------ fwd + adjoint
        nb = 16384
        xa = x_all[: nb * n].view(nb, n)
        ya = y_all[: nb * n].view(nb, n)
        za = torch.empty_like(xa)
        pa = api.Plan(n, nb, -1)
        ms_f = time_launches(lambda: pa.execute(xa, ya), args.steps, args.warmup, torch)

        def fa():
            pa.execute(xa, ya)
            pa.adjoint(ya, za)
        ms_fa = time_launches(fa, args.steps, args.warmup, torch)
        b1 = 16.0 * nb * n
        w = torch.from_numpy(synth.uniform_weights(synth.SEED_AUTOGRAD, (nb, n))).to(dev)
        xg = xa.clone().requires_grad_(True)

        def step():
            xg.grad = None
            yy = api.fft_differentiable(xg)
            loss = (w * (yy.real ** 2 + yy.imag ** 2)).sum()
            loss.backward()
        ms_step = time_launches(step, max(20, args.steps // 5), 3, torch)
        out["fwd_adjoint"] = {
            "workload": "N=2048 batch 16384 (256 MiB per pass)",
            "fwd_ms": round(ms_f, 5), "fwd_GBps": round(b1 / (ms_f * 1e-3) / 1e9, 1),
            "fwd_adj_ms": round(ms_fa, 5), "fwd_adj_GBps": round(2 * b1 / (ms_fa * 1e-3) / 1e9, 1),
            "ratio_fwd_adj_over_fwd": round(ms_fa / ms_f, 3),
            "autograd_step_ms": round(ms_step, 5),
        }
        log(f"[bench] fwd+adj {out['fwd_adjoint']}")
        del xg, w

        # ------------------------------------------------------------ sweep
        if not args.no_sweep:
            sweep = []
            for L in range(1, 12):
                nn = 1 << L
                bb = total // nn
                xs, ys = x_all.view(bb, nn), y_all.view(bb, nn)
                row = {"n": nn, "batch": bb}
                for sign, nm in ((-1, "fwd"), (1, "inv")):
                    p = api.Plan(nn, bb, sign)
                    m = time_launches(lambda: p.execute(xs, ys), max(20, args.steps // 4), 5, torch)
                    row[f"{nm}_us"] = round(m * 1e3, 2)
                    row[f"{nm}_GBps"] = round(bytes_alg / (m * 1e-3) / 1e9, 1)
                    row[f"{nm}_GFLOPs"] = round(5.0 * nn * L * bb / (m * 1e-3) / 1e9, 1)
                    d = p.describe()
                    row["ept"], row["wg"] = d["ept"], d["wg"]
                    p.close()
                sweep.append(row)
                log(f"[bench] sweep {row}")
            out["sweep"] = sweep

    # ---------------------------------------------------------------- cpu baseline
    if not args.no_cpu:
        log("[bench] timing the FP64 CPU oracle")
        out["cpu_baseline"] = cpu_baseline(n)
        log(f"[bench] cpu {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
