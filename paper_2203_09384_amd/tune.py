"""Autotuner: times every compiled kernel variant and writes the tuned table.

For the batched FP32 path it times, per length N, each (elements per thread,
workgroup size) variant compiled into libmifft.so on a batch of `total`
elements, and keeps the fastest.  For ragged batches it picks, per length,
the elements-per-thread of the ragged kernel and the workgroup size of
the launch, timing one graph-free launch over a seeded ragged batch.  Real-input plans (R2C and C2R) are tuned per half length on the
sum of both directions' times.  The result is a text table ("c32 <log2n>
<ept> <wg> <variant>", "r32 <log2(n/2)> <ept> <wg> <variant>" and
"ragged <log2n> <ept>" / "ragged_wg <wg> <ctas_per_cu>" lines) that the library reads
from the file named by MIFFT_TUNE_TABLE, plus a JSON record of every
timing.

    python -m paper_2203_09384_amd.tune --out tune_gfx950.txt
"""
from __future__ import annotations

import argparse
import json
import math
import sys

EPTS = (2, 4, 8, 16)
WGS = (64, 128, 256, 512, 1024)
VARIANTS = tuple(range(10)) + (11, 12)  # 9: four-step, lengths above 2048 only; 11, 12: staged, n <= 64


def _time(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        fn()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune_c32(total: int = 1 << 26, steps: int = 30, warmup: int = 5, log2ns=range(1, 15), log=print):
    import torch
    from . import api, synth
    from .native import MifftError
    x = torch.from_numpy(synth.uniform_complex(synth.SEED_PLAIN, (total,), key=(0,))).cuda()
    y = torch.empty_like(x)
    best, record = {}, []
    for L in log2ns:
        n = 1 << L
        b = total // n
        xs, ys = x[: b * n].view(b, n), y[: b * n].view(b, n)
        for ept in EPTS:
            for wg in WGS:
                for var in VARIANTS:
                    if var == 9 and (L <= 11 or ept != EPTS[0] or wg != WGS[0]):
                        continue
                    try:
                        p = api.Plan(n, b, -1, ept=ept, wg=wg, variant=var)
                    except MifftError:
                        continue
                    ms = _time(lambda: p.execute(xs, ys), steps, warmup, torch)
                    gbps = 16.0 * b * n / (ms * 1e-3) / 1e9
                    rec = {"n": n, "ept": ept, "wg": wg, "variant": var, "us": round(ms * 1e3, 2),
                           "GBps": round(gbps, 1), "grid": p.describe()["grid"]}
                    record.append(rec)
                    log(f"[tune] {rec}")
                    if L not in best or ms < best[L][3]:
                        best[L] = (ept, wg, var, ms)
                    p.close()
    return best, record


def tune_loss(total: int = 1 << 25, steps: int = 30, warmup: int = 5, log2ns=range(1, 12), log=print):
    """Fused loss-gradient kernel: every compiled (ept, wg) shape, selected
    through a plan forced to that shape (any compiled FP32 variant of it),
    timed on `total` elements."""
    import torch
    from . import api, synth
    from .native import MifftError
    x = torch.from_numpy(synth.uniform_complex(synth.SEED_AUTOGRAD, (total,), key=(0,))).cuda()
    w = torch.from_numpy(synth.uniform_weights(synth.SEED_AUTOGRAD, (total,))).cuda()
    g = torch.empty_like(x)
    best, record = {}, []
    for L in log2ns:
        n = 1 << L
        b = total // n
        xs, ws, gs = x[: b * n].view(b, n), w[: b * n].view(b, n), g[: b * n].view(b, n)
        lv = torch.empty(b, dtype=torch.float32, device=x.device)
        for ept in EPTS:
            for wg in (64, 128, 256):
                p = None
                for var in (0, 2, 1, 6, 3):
                    try:
                        p = api.Plan(n, b, -1, ept=ept, wg=wg, variant=var)
                        break
                    except MifftError:
                        continue
                if p is None:
                    continue
                try:
                    ms = _time(lambda: p.loss_grad(xs, ws, gs, lv), steps, warmup, torch)
                except MifftError:
                    p.close()
                    continue
                rec = {"n": n, "ept": ept, "wg": wg, "us": round(ms * 1e3, 2),
                       "GBps": round(20.0 * b * n / (ms * 1e-3) / 1e9, 1)}
                record.append(rec)
                log(f"[tune-loss] {rec}")
                if L not in best or ms < best[L][2]:
                    best[L] = (ept, wg, ms)
                p.close()
    return best, record


REAL_EPTS = (1, 2, 4, 8, 16)
REAL_VARIANTS = (0, 2, 3, 6, 7)


def tune_real(total: int = 1 << 27, steps: int = 30, warmup: int = 5, log2ns=range(2, 16), log=print):
    """Real-input plans: every compiled (ept, wg, variant) of the half-length
    transform, timed as R2C plus C2R over `total` float32 reals."""
    import torch
    from . import api, synth
    from .native import MifftError
    xr = torch.from_numpy(synth.uniform_real(synth.SEED_REAL, (total,), key=(0,))).cuda()
    back = torch.empty_like(xr)
    best, record = {}, []
    for L in log2ns:
        n = 1 << L
        b = total // n
        xs, bs = xr[: b * n].view(b, n), back[: b * n].view(b, n)
        bins = torch.empty(b, n // 2 + 1, dtype=torch.complex64, device=xr.device)
        for ept in REAL_EPTS:
            for wg in WGS:
                for var in REAL_VARIANTS:
                    try:
                        pf = api.Plan(n, b, -1, "r32", ept=ept, wg=wg, variant=var)
                        pi = api.Plan(n, b, +1, "r32", ept=ept, wg=wg, variant=var)
                    except MifftError:
                        continue
                    ms_f = _time(lambda: pf.execute(xs, bins), steps, warmup, torch)
                    ms_i = _time(lambda: pi.execute(bins, bs), steps, warmup, torch)
                    alg = b * (4.0 * n + 8.0 * (n // 2 + 1))
                    rec = {"n": n, "ept": ept, "wg": wg, "variant": var, "r2c_us": round(ms_f * 1e3, 2),
                           "c2r_us": round(ms_i * 1e3, 2), "r2c_GBps": round(alg / (ms_f * 1e-3) / 1e9, 1),
                           "c2r_GBps": round(alg / (ms_i * 1e-3) / 1e9, 1)}
                    record.append(rec)
                    log(f"[tune-real] {rec}")
                    if L - 1 not in best or ms_f + ms_i < best[L - 1][3]:
                        best[L - 1] = (ept, wg, var, ms_f + ms_i)
                    pf.close()
                    pi.close()
        del bins
    return best, record


def tune_ragged(count: int = 4096, iters: int = 300, log=print):
    """Per-length elements per thread and the workgroup size of the ragged
    kernel, by coordinate descent on one seeded ragged batch
    (lengths 2^3..2^11), timing one launch per call."""
    import numpy as np
    import torch
    from . import api, synth
    from .native import MifftError
    lengths = synth.ragged_lengths(synth.SEED_RAGGED, count, 3, 11)
    off = synth.offsets_from_lengths(lengths)
    x = torch.from_numpy(synth.uniform_complex(synth.SEED_RAGGED, (int(off[-1]),), key=(1,))).cuda()
    y = torch.empty_like(x)

    def cost(table, wg):
        try:
            p = api.RaggedPlan(off, -1, ept_by_log2n=table, wg=wg)
        except MifftError:
            return float("inf")
        ms = min(_time(lambda: p.execute(x, y), iters, 20, torch) for _ in range(2))
        p.close()
        return ms

    record, best = [], None
    # a length's threads (at most 16 points each) must fit the workgroup
    for wg in [w for w in (64, 128, 256) if int(lengths.max()) // 16 <= w]:
        table = [0, 2, 4, 8, 4, 4, 4, 8, 8, 8, 8, 8]
        cur = cost(table, wg)
        for _ in range(2):
            for L in range(3, 12):
                for ept in (4, 8, 16):
                    if ept > (1 << L) or ept == table[L]:
                        continue
                    trial = list(table)
                    trial[L] = ept
                    c = cost(trial, wg)
                    if c < cur:
                        cur, table = c, trial
        rec = {"wg": wg, "ept_by_log2n": table, "us": round(cur * 1e3, 2)}
        record.append(rec)
        log(f"[tune-ragged] {rec}")
        if best is None or cur < best[2]:
            best = (wg, table, cur)
    return {"wg": best[0], "ctas_per_cu": 0, "ept": {L: best[1][L] for L in range(1, 12) if best[1][L]},
            "us": round(best[2] * 1e3, 2)}, record


def write_table(path: str, best_c32: dict, ragged: dict | None = None, best_r32: dict | None = None,
                best_loss: dict | None = None):
    with open(path, "w") as f:
        f.write("# mifft tuned variants for gfx950 (written by paper_2203_09384_amd.tune)\n")
        for L in sorted(best_c32):
            ept, wg, var, ms = best_c32[L]
            f.write(f"c32 {L} {ept} {wg} {var}  # {ms * 1e3:.2f} us\n")
        for L in sorted(best_r32 or {}):
            ept, wg, var, ms = best_r32[L]
            f.write(f"r32 {L} {ept} {wg} {var}  # r2c + c2r {ms * 1e3:.2f} us\n")
        for L in sorted(best_loss or {}):
            ept, wg, ms = best_loss[L]
            f.write(f"loss {L} {ept} {wg}  # fused loss + gradient {ms * 1e3:.2f} us\n")
        if ragged:
            for L in sorted(ragged.get("ept", {})):
                f.write(f"ragged {L} {ragged['ept'][L]}\n")
            if "wg" in ragged:
                f.write(f"ragged_wg {ragged['wg']} {ragged.get('ctas_per_cu', 0)}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tune_gfx950.txt")
    ap.add_argument("--json", default=None)
    ap.add_argument("--total-log2", type=int, default=26)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--skip-c32", action="store_true")
    ap.add_argument("--skip-ragged", action="store_true")
    ap.add_argument("--skip-real", action="store_true")
    ap.add_argument("--skip-loss", action="store_true")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    best, rec = ({}, []) if args.skip_c32 else tune_c32(1 << args.total_log2, args.steps, log=log)
    rbest, rrec = (None, []) if args.skip_ragged else tune_ragged(log=log)
    real_best, real_rec = ({}, []) if args.skip_real else tune_real(1 << (args.total_log2 + 1), args.steps,
                                                                      log=log)
    loss_best, loss_rec = ({}, []) if args.skip_loss else tune_loss(1 << (args.total_log2 - 1), args.steps, log=log)
    write_table(args.out, best, rbest, real_best, loss_best)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"c32": rec, "best": {L: best[L][:3] for L in best}, "ragged": rrec,
                       "ragged_best": rbest, "real": real_rec,
                       "real_best": {L: real_best[L][:3] for L in real_best}, "loss": loss_rec,
                       "loss_best": {L: loss_best[L][:2] for L in loss_best}}, f, indent=1)
    print(json.dumps({"c32": {L: best[L][:3] for L in best}, "ragged": rbest,
                      "r32": {L: real_best[L][:3] for L in real_best},
                      "loss": {L: loss_best[L][:2] for L in loss_best}}))


if __name__ == "__main__":
    main()
