#!/usr/bin/env python3
"""Benchmark of the batched FP32 C2C FFT on one MI355X.

Headline workload: forward FFT, N = 2048, batch 32768 (2^26 complex64
elements: 512 MiB read + 512 MiB written per step), inputs resident in HBM.
One step = one fft_execute of that batch.  Also measured in the same run:
the forward + adjoint pair of the differentiable FFT (N = 2048, batch
16384), the per-N sweep (every N = 2..2048 at 2^26 elements, forward and
inverse), a plain 512 MiB copy kernel as the practical bandwidth ceiling,
the ragged batch (4096 mixed lengths, one launch vs per-length
launches), and the FP64 CPU oracle on a bounded sample (cpu_baseline).

Prints ONE JSON line.  Times come from HIP events recorded on the stream
the kernels are launched on (torch's current stream).
"""
import argparse
import ctypes
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "FP32 C2C FFT GFLOP/s (5NlogN) & HBM GB/s at N=2048; fwd+adjoint vs plain fwd"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fft_c32_n2048_b32768.json")
COPY_LIB = os.path.join(ROOT, "paper_2203_09384_amd", "libstreamcopy.so")


def tune_table_id():
    """Which variant table the library plans with: the built-in one, or a
    hash of the file named by MIFFT_TUNE_TABLE."""
    path = os.environ.get("MIFFT_TUNE_TABLE", "")
    if not path:
        return "builtin"
    with open(path, "rb") as f:
        return "file:" + hashlib.sha256(f.read()).hexdigest()[:16]


def read_clocks():
    """Current GPU clocks as rocm-smi reports them (another process; no
    effect on the run), or the error."""
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=30)
        d = json.loads(r.stdout)
        card = d.get("card0") or next(iter(d.values()))
        return {k.strip(" :"): v for k, v in card.items() if "clk" in k.lower()}
    except Exception as e:  # noqa: BLE001
        return {"error": f"{type(e).__name__}: {str(e)[:120]}"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_name(d):
    """Name of the kernel template instance a plan launches."""
    L = int(math.log2(d["n"]))
    e = int(math.log2(d["ept"]))
    if d["variant"] == 0:
        return f"k_fft_c32<{L}, {e}, {d['wg']}, {d['sign']}>"
    v = d["variant"] - 1
    wave = v >= 4
    v %= 4
    return f"k_fft_c32_v2<{L}, {e}, {d['wg']}, {d['sign']}, {v % 2}, {v // 2}, {str(wave).lower()}>"


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


def cpu_baseline(n, batch, budget_s=12.0):
    """FP64 oracle on a bounded sample of the headline workload: chunks of
    the same seeded N=2048 batch, repeated until about budget_s seconds."""
    import numpy as np
    import oracle
    from paper_2203_09384_amd import synth
    threads = oracle.default_threads()
    chunk = min(batch, 4096)
    x = synth.uniform_complex(synth.SEED_PLAIN, (chunk * n,), key=(0,)).reshape(chunk, n).astype(np.complex128)
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.forward(x, threads=threads)
        done += chunk
        dt = time.perf_counter() - t0
        if dt >= budget_s or done >= 64 * batch:
            break
    flops = 5.0 * n * math.log2(n) * done
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} forward transforms of N={n} (the first {chunk} transforms of the headline "
                      f"batch, repeated; FP64 recursive radix-2 on {threads} threads, {dt:.1f} s)",
            "seconds": round(dt, 2), "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def half_accuracy(samples):
    """Per-transform relative L2 of the FP16/BF16 results against the FP64
    oracle on the stored input (and on the raw FP64 draw), per dtype and
    input class, over the sampled transforms the half section kept."""
    import numpy as np
    import oracle
    res = {}
    for (dt, cls), (x_stored, x_raw, y) in samples.items():
        def worst(ref):
            return float(np.max(np.linalg.norm(y - ref, axis=-1) / np.linalg.norm(ref, axis=-1)))
        res.setdefault(dt, {})[cls] = {"max_rel_l2_vs_stored_input": worst(oracle.forward(x_stored)),
                                       "max_rel_l2_vs_raw_draw": worst(oracle.forward(x_raw)),
                                       "transforms": int(y.shape[0])}
    return res


def time_rotating(fns, steps, warmup, torch):
    """Average ms per call over `steps` back-to-back calls that cycle
    through fns (one per buffer set), as time_launches."""
    i = [0]

    def step():
        fns[i[0] % len(fns)]()
        i[0] += 1
    return time_launches(step, steps, warmup, torch)


HALF_SETS = 4  # input/output buffer sets cycled by the FP16/BF16 timing


def bench_half(api, synth, torch, dev, steps, ms_fp32, x_all, samples=None):
    """FP16 / BF16 block-floating-point forward FFT, N = 2048, batch 32768,
    against the FP32 kernel at the same shape (ms_fp32), for both input
    classes (re, im uniform[-1, 1); magnitude log-uniform in [1e-3, 1e3] with
    uniform phase).  The input is 256 MiB, which the 256 MB last-level
    cache can partly keep between launches: the reported time cycles
    through HALF_SETS buffer sets (1 GiB of inputs), so each launch streams
    from HBM; the time on one repeated set is reported beside it.
    Sampled transforms (inputs as stored, raw draws and de-scaled outputs)
    go to `samples` for the accuracy check against the FP64 oracle,
    outside the timed region."""
    import numpy as np
    n, batch = 2048, 32768
    res = {"workload": "C2C forward FFT, N=2048, batch 32768, FP16/BF16 storage (4 B per element), "
                       "per-transform int32 exponents, radix-16 passes on MFMA; classes: uniform[-1,1) re/im, "
                       "log-uniform magnitude 1e-3..1e3 with uniform phase",
           "timing": f"launches cycle through {HALF_SETS} input/output buffer sets (no reuse of the "
                     "256 MiB input from the last-level cache); us_same_buffers: one set repeated"}
    rng = np.random.default_rng(20220320)
    idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 126)]))
    for dt, tdt in (("c16", torch.float16), ("cbf16", torch.bfloat16)):
        res[dt] = {}
        for cls in ("uniform", "loguniform"):
            if cls == "uniform":
                xc = x_all.view(batch, n)
                raw = None
            else:
                raw = synth.log_uniform_polar(synth.SEED_HALF, (batch, n), key=(1, 1))
                xc = torch.from_numpy(raw.astype(np.complex64)).to(dev)
            xh = [torch.view_as_real(xc).to(tdt).contiguous() for _ in range(HALF_SETS)]
            yh = [torch.empty_like(xh[0]) for _ in range(HALF_SETS)]
            ex = [torch.empty(batch, dtype=torch.int32, device=dev) for _ in range(HALF_SETS)]
            p = api.Plan(n, batch, -1, dtype=dt)
            m = time_rotating([(lambda i=i: p.execute_scaled(xh[i], out=yh[i], out_exp=ex[i]))
                               for i in range(HALF_SETS)], steps, 20, torch)
            m1 = time_launches(lambda: p.execute_scaled(xh[0], out=yh[0], out_exp=ex[0]), steps, 20, torch)
            alg = 8.0 * n * batch + 4.0 * batch
            res[dt][cls] = {"us": round(m * 1e3, 2), "GBps": round(alg / (m * 1e-3) / 1e9, 1),
                            "GFLOPs": round(5.0 * n * 11 * batch / (m * 1e-3) / 1e9, 1),
                            "speedup_vs_fp32": round(ms_fp32 / m, 3),
                            "us_same_buffers": round(m1 * 1e3, 2)}
            if samples is not None:
                it = torch.from_numpy(idx).to(dev)
                xs = xh[0][it].float().cpu().numpy().astype(np.float64)
                ys = yh[0][it].float().cpu().numpy().astype(np.float64)
                e = np.exp2(ex[0][it].cpu().numpy().astype(np.float64))[:, None]
                x_raw = (x_all.view(batch, n)[it].cpu().numpy().astype(np.complex128) if raw is None
                         else raw[idx])
                samples[(dt, cls)] = (xs[..., 0] + 1j * xs[..., 1], x_raw, (ys[..., 0] + 1j * ys[..., 1]) * e)
            p.close()
            del xh, yh, ex
        # the headline figures of this dtype: the uniform class
        res[dt].update({k: res[dt]["uniform"][k] for k in ("us", "GBps", "GFLOPs", "speedup_vs_fp32")})
    return res


def bench_copy(torch, x_all, y_all, steps, warmup):
    """The practical HBM ceiling: a hand-written 512 MiB streaming copy
    (16-byte nontemporal loads and stores, several workgroup shapes; the
    best is reported), and torch's elementwise copy for reference."""
    lib = ctypes.CDLL(COPY_LIB)
    lib.stream_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    lib.stream_copy_shape.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    nbytes = x_all.numel() * x_all.element_size()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    shapes = {}
    for i in range(lib.stream_copy_shapes()):
        wg, k = ctypes.c_int(), ctypes.c_int()
        lib.stream_copy_shape(i, ctypes.byref(wg), ctypes.byref(k))

        def run():
            rc = lib.stream_copy(ctypes.c_void_p(x_all.data_ptr()), ctypes.c_void_p(y_all.data_ptr()), nbytes, i, st)
            if rc != 0:
                raise RuntimeError(f"stream_copy shape {i} failed: {rc}")
        ms = time_launches(run, steps, warmup, torch)
        shapes[f"wg{wg.value}_k{k.value}"] = round(2.0 * nbytes / (ms * 1e-3) / 1e9, 1)
    ms_t = time_launches(lambda: torch.mul(x_all, 1.0, out=y_all), steps, warmup, torch)
    assert torch.equal(x_all, y_all)
    return {"GBps": max(shapes.values()), "shapes_GBps": shapes,
            "torch_elementwise_GBps": round(2.0 * nbytes / (ms_t * 1e-3) / 1e9, 1),
            "bytes_each_way": nbytes,
            "kernel": "k_stream_copy<WG, K>: K 16-byte nontemporal vectors per thread, 1 KiB per wave instruction"}


def bench_real(api, torch, dev, steps, x_all):
    """Real-input transforms, n = 2048, batch 65536: R2C (512 MiB of float32
    reals in, 65536 x 1025 complex64 bins out) and C2R back."""
    n, batch = 2048, 65536
    xr = torch.view_as_real(x_all).view(batch, n)
    bins = torch.empty(batch, n // 2 + 1, dtype=torch.complex64, device=dev)
    back = torch.empty(batch, n, dtype=torch.float32, device=dev)
    alg = batch * (4.0 * n + 8.0 * (n // 2 + 1))
    res = {"workload": "real-input FFT, n=2048, batch 65536: R2C float32 (512 MiB) -> 1025 complex64 "
                       "bins per transform, and C2R back; one fused kernel each (half-length complex "
                       "FFT plus the even/odd split)"}
    for nm, sign, a, b in (("r2c", -1, xr, bins), ("c2r", +1, bins, back)):
        p = api.Plan(n, batch, sign, dtype="r32")
        m = time_launches(lambda: p.execute(a, b), steps, 10, torch)
        d = p.describe()
        res[nm] = {"us": round(m * 1e3, 2), "GBps": round(alg / (m * 1e-3) / 1e9, 1),
                   "GFLOPs_2.5nlogn": round(2.5 * n * 11 * batch / (m * 1e-3) / 1e9, 1),
                   "ept": d["ept"], "wg": d["wg"], "variant": d["variant"]}
        p.close()
    res["algorithmic_bytes_per_launch"] = alg
    del bins, back
    # above 2^15: four-step half-length transform + split pass (workspace)
    nl, bl = 1 << 20, 64
    xl = torch.view_as_real(x_all).view(-1)[: nl * bl].view(bl, nl)
    binl = torch.empty(bl, nl // 2 + 1, dtype=torch.complex64, device=dev)
    p = api.Plan(nl, bl, -1, dtype="r32")
    m = time_launches(lambda: p.execute(xl, binl), max(20, steps // 4), 5, torch)
    alg_l = bl * (4.0 * nl + 8.0 * (nl // 2 + 1))
    res["r2c_n2^20_batch64"] = {"us": round(m * 1e3, 2), "GBps_algorithmic": round(alg_l / (m * 1e-3) / 1e9, 1),
                                "passes_over_hbm": 3}
    p.close()
    del binl
    return res


def bench_nd(api, torch, steps, x_all, y_all):
    """2D 2048 x 2048 (batch 16), 128 x 128 and 64 x 64, and 3D 128^3
    (batch 32) and 16^3 (batch 16384) forward transforms, 2^26 complex64
    elements each way; one HBM pass per axis, or one in all for arrays that
    fit one workgroup's LDS."""
    res = {"workload": "multidimensional C2C forward FFT, 2^26 complex64 elements (512 MiB in + 512 MiB out); "
                       "the last axis through the batched kernels, each other axis one in-place tiled pass"}
    for name, shape, batch in (("2d_2048x2048", (2048, 2048), 16), ("2d_128x128", (128, 128), 4096),
                               ("2d_64x64", (64, 64), 16384), ("3d_128x128x128", (128, 128, 128), 32),
                               ("3d_16x16x16", (16, 16, 16), 16384)):
        p = api.PlanND(shape, batch, -1)
        xs = x_all.view((batch,) + shape)
        ys = y_all.view((batch,) + shape)
        m = time_launches(lambda: p.execute(xs, ys), max(20, steps // 2), 5, torch)
        elems = batch
        for d in shape:
            elems *= d
        variant = p.describe()["variant"]
        passes = 1 if variant == 13 else len(shape) - 1 if variant == 10 else len(shape)
        res[name] = {"us": round(m * 1e3, 2), "passes_over_hbm": passes,
                     "GBps_algorithmic": round(16.0 * elems / (m * 1e-3) / 1e9, 1),
                     "GBps_actual_passes": round(16.0 * passes * elems / (m * 1e-3) / 1e9, 1),
                     "GFLOPs": round(5.0 * elems * math.log2(elems // batch) / (m * 1e-3) / 1e9, 1)}
        p.close()
    return res


def bench_ragged(api, synth, torch, dev, iters):
    """One launch over 4096 mixed-length transforms (eager and
    graph-replayed) against per-length plain launches (eager and in one
    graph), the transforms pre-grouped by length outside the timed region."""
    import numpy as np
    lengths = synth.ragged_lengths(synth.SEED_RAGGED, 4096, 3, 11)
    off = synth.offsets_from_lengths(lengths)
    total = int(off[-1])
    x = torch.from_numpy(synth.uniform_complex(synth.SEED_RAGGED, (total,), key=(1,))).to(dev)
    y = torch.empty_like(x)
    rp = api.RaggedPlan(off, -1)
    desc = rp.describe()
    t_eager = time_launches(lambda: rp.execute(x, y), iters, 50, torch)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rp.execute(x, y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        rp.execute(x, y)
    t_graph = time_launches(g.replay, iters, 50, torch)
    # per-length batches, grouped once (untimed)
    groups = []
    for L in range(3, 12):
        idx = np.nonzero(lengths == (1 << L))[0]
        if len(idx) == 0:
            continue
        n = 1 << L
        cols = (off[idx][:, None] + np.arange(n)[None, :]).reshape(-1)
        xs = x[torch.from_numpy(cols).to(dev)].view(len(idx), n).contiguous()
        groups.append((api.Plan(n, len(idx), -1), xs, torch.empty_like(xs)))

    def per_length():
        for p, xs, ys in groups:
            p.execute(xs, ys)
    t_pl = time_launches(per_length, iters, 50, torch)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        per_length()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g2):
        per_length()
    t_pl_graph = time_launches(g2.replay, iters, 50, torch)
    # the same two paths with REPS batches captured in one graph: per-batch
    # GPU time once the graph launch itself is amortised
    reps = 20
    g3, g4 = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g3):
        for _ in range(reps):
            rp.execute(x, y)
    with torch.cuda.graph(g4):
        for _ in range(reps):
            per_length()
    t_graph_rep = time_launches(g3.replay, max(10, iters // reps), 5, torch) / reps
    t_pl_graph_rep = time_launches(g4.replay, max(10, iters // reps), 5, torch) / reps
    flops = float(np.sum(5.0 * lengths * np.log2(lengths)))
    bytes_ = 16.0 * total
    us = lambda ms: round(ms * 1e3, 2)
    return {
        "workload": "4096 FP32 C2C forward transforms, N=2^L with L uniform on 3..11 (seeded), "
                    f"{total} elements packed with int64 offsets",
        "persistent_eager_us": us(t_eager), "persistent_graph_us": us(t_graph),
        "per_length_eager_us": us(t_pl), "per_length_graph_us": us(t_pl_graph),
        "launches_per_length_path": len(groups),
        "speedup_vs_per_length_eager": round(t_pl / t_eager, 2),
        "speedup_graph_vs_per_length_graph": round(t_pl_graph / t_graph, 2),
        "graph_of_20_batches": {"persistent_us_per_batch": us(t_graph_rep),
                                "per_length_us_per_batch": us(t_pl_graph_rep),
                                "speedup": round(t_pl_graph_rep / t_graph_rep, 2)},
        "persistent_graph_GFLOPs": round(flops / (t_graph * 1e-3) / 1e9, 1),
        "persistent_graph_effective_GBps": round(bytes_ / (t_graph * 1e-3) / 1e9, 1),
        "note": "about 30 MB moved: cache-resident, so effective GB/s is not an HBM figure",
        "plan": {k: desc[k] for k in ("wg", "grid", "tiles", "lds_bytes", "ept_by_log2n")},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["headline", "half", "loss", "copy", "large", "nd"], default=None,
                    help="time one section only (for profiler runs); 'headline' with --with-copy also runs "
                         "the streaming copy (counter calibration)")
    ap.add_argument("--only-headline", action="store_true", help="same as --only headline")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --only SECTION: also run the 512 MiB streaming copy (counter calibration)")
    args = ap.parse_args()
    if args.only_headline:
        args.only = "headline"
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the batched transforms are independent, so the path "
              f"has no multi-GPU step to run here (got --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_09384_amd import api, synth
    from paper_2203_09384_amd.profiling import kernel_hash

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
    only = args.only
    if only in ("half", "loss", "copy", "large", "nd"):
        run_section(only, args, api, synth, torch, dev, x_all, y_all)
        return
    plan = api.Plan(n, batch, -1)
    desc = plan.describe()
    log(f"[bench] headline plan {desc}")
    # rocm-smi is a separate program; under a profiler (the --only runs) its
    # interpreter would start inside the profiled process tree, so skip it
    clocks_before = read_clocks() if only is None else {"skipped": "single-section run"}
    # settle clocks: about half a second of the same kernel before timing
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        for _ in range(20):
            plan.execute(x, y)
        torch.cuda.synchronize()
    ms = time_launches(lambda: plan.execute(x, y), args.steps, args.warmup, torch)
    clocks_after = read_clocks() if only is None else {"skipped": "single-section run"}
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
                   "variant": desc["variant"], "grid": desc["grid"],
                   "radices": desc["radices"], "seed": synth.SEED_PLAIN},
    }
    # measured HBM traffic, when profiles/ holds counters taken for this very
    # kernel instance, these sources and this variant table
    traffic = None
    khash, kname, table = kernel_hash(), kernel_name(desc), tune_table_id()
    traffic_note = "no counter record"
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        key = (tr.get("kernel_instance"), tr.get("kernel_hash"), tr.get("tune_table"))
        if key == (kname, khash, table):
            traffic = tr.get("bytes_per_launch")
            traffic_note = "counters of this kernel instance, sources and variant table"
        else:
            traffic_note = f"counter record is for {key}, not ({kname}, {khash}, {table})"
    out["roofline"] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic,
                       "kernel": kname, "kernel_hash": khash, "tune_table": table,
                       "traffic_note": traffic_note, "algorithmic_bytes_per_launch": bytes_alg}
    out["headline_distribution"] = per_call_distribution(lambda: plan.execute(x, y), 50, torch)
    out["gflops_fwd_2048"] = round(gflops, 1)
    out["gbps_fwd_2048"] = round(gbps, 1)
    out["clocks"] = {"before_headline": clocks_before, "after_headline": clocks_after}
    out["host"] = {"cpu_model": cpu_model(), "cpus": os.cpu_count(), "gpu": props.name,
                   "arch": getattr(props, "gcnArchName", ""), "cus": props.multi_processor_count}

    if only == "headline" and args.with_copy:
        bench_copy(torch, x_all, y_all, args.steps, args.warmup)
    half_samples = {}

    if only is None:
        # ------------------------------------------------------------ copy ceiling
        copy = bench_copy(torch, x_all, y_all, args.steps, args.warmup)
        out["copy_ceiling_GBps"] = copy["GBps"]
        out["copy_ceiling"] = copy
        log(f"[bench] copy 512 MiB: {copy}")

        # ------------------------------------------------------------ fwd + adjoint
        out["fwd_adjoint"] = bench_fwd_adjoint(api, synth, torch, dev, args, x_all, y_all)
        log(f"[bench] fwd+adj {out['fwd_adjoint']}")

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

        # ------------------------------------------------------------ lengths above 2048
        out["large_n"] = bench_large(api, torch, args, x_all, y_all)
        log(f"[bench] large {out['large_n']}")

        # ------------------------------------------------------------ FP16 / BF16
        out["half"] = bench_half(api, synth, torch, dev, args.steps, ms, x_all, half_samples)
        log(f"[bench] half {out['half']}")

        # ------------------------------------------------------------ real input
        out["real"] = bench_real(api, torch, dev, args.steps, x_all)
        log(f"[bench] real {out['real']}")

        # ------------------------------------------------------------ multidimensional
        out["nd"] = bench_nd(api, torch, args.steps, x_all, y_all)
        log(f"[bench] nd {out['nd']}")

        # ------------------------------------------------------------ ragged
        out["ragged"] = bench_ragged(api, synth, torch, dev, max(200, args.steps * 5))
        log(f"[bench] ragged {out['ragged']}")

    # ---------------------------------------------------------------- cpu baseline
    # the FP64 oracle on the host: its throughput on a bounded sample of the
    # headline workload, and the accuracy of the sampled FP16/BF16 results
    if not args.no_cpu:
        log("[bench] timing the FP64 CPU oracle")
        out["cpu_baseline"] = cpu_baseline(n, batch)
        log(f"[bench] cpu {out['cpu_baseline']}")
        if half_samples:
            out["half"]["accuracy_vs_fp64_oracle"] = half_accuracy(half_samples)
            log(f"[bench] half accuracy {out['half']['accuracy_vs_fp64_oracle']}")
    print(json.dumps(out), flush=True)


def bench_fwd_adjoint(api, synth, torch, dev, args, x_all, y_all):
    """The differentiable FFT at N = 2048, batch 16384: forward, forward +
    adjoint, the autograd step, and the fused loss-gradient kernel."""
    n, nb = 2048, 16384
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
    lossv = torch.empty(nb, dtype=torch.float32, device=dev)
    ms_fused = time_launches(lambda: pa.loss_grad(xa, w, za, lossv), args.steps, args.warmup, torch)

    def fused_step():
        xg.grad = None
        api.weighted_power_loss(xg, w).backward()
    ms_fused_step = time_launches(fused_step, max(20, args.steps // 5), 3, torch)
    return {
        "workload": "N=2048 batch 16384 (256 MiB per pass)",
        "fwd_ms": round(ms_f, 5), "fwd_GBps": round(b1 / (ms_f * 1e-3) / 1e9, 1),
        "fwd_adj_ms": round(ms_fa, 5), "fwd_adj_GBps": round(2 * b1 / (ms_fa * 1e-3) / 1e9, 1),
        "ratio_fwd_adj_over_fwd": round(ms_fa / ms_f, 3),
        "autograd_step_ms": round(ms_step, 5),
        "fused_loss_grad_ms": round(ms_fused, 5),
        "fused_loss_grad_GBps": round((20.0 * nb * n + 4.0 * nb) / (ms_fused * 1e-3) / 1e9, 1),
        "fused_autograd_step_ms": round(ms_fused_step, 5),
        "note": "fused: loss[b] = sum w|Fx|^2 and grad = F^H(2w Fx) in one kernel, 20 B per element",
    }


def bench_large(api, torch, args, x_all, y_all):
    """Lengths above 2048 at 2^26 elements: one pass up to 2^14, the
    two-pass four-step above."""
    total = x_all.numel()
    large = []
    for L in (12, 14, 16, 20):
        nn = 1 << L
        bb = total // nn
        p = api.Plan(nn, bb, -1)
        m = time_launches(lambda: p.execute(x_all.view(bb, nn), y_all.view(bb, nn)),
                          max(20, args.steps // 4), 5, torch)
        passes = 2 if p.describe()["variant"] == 9 else 1
        large.append({"n": nn, "batch": bb, "us": round(m * 1e3, 2),
                      "GFLOPs": round(5.0 * nn * L * bb / (m * 1e-3) / 1e9, 1),
                      "GBps_algorithmic": round(16.0 * total / (m * 1e-3) / 1e9, 1),
                      "GBps_actual_passes": round(16.0 * passes * total / (m * 1e-3) / 1e9, 1),
                      "passes_over_hbm": passes})
        p.close()
    return large


def run_section(only, args, api, synth, torch, dev, x_all, y_all):
    """One section alone, for profiler runs; prints its JSON."""
    res = {"section": only}
    if only == "half":
        res["half"] = bench_half(api, synth, torch, dev, args.steps, float("nan"), x_all)
    elif only == "loss":
        res["fwd_adjoint"] = bench_fwd_adjoint(api, synth, torch, dev, args, x_all, y_all)
    elif only == "copy":
        res["copy"] = bench_copy(torch, x_all, y_all, args.steps, args.warmup)
    elif only == "large":
        res["large_n"] = bench_large(api, torch, args, x_all, y_all)
    elif only == "nd":
        res["nd"] = bench_nd(api, torch, args.steps, x_all, y_all)
    if args.with_copy and only != "copy":  # counter calibration in the same run
        res["copy"] = bench_copy(torch, x_all, y_all, args.steps, args.warmup)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
