"""Benchmark of the FastCauchyRegression hot path on one MI355X.

A step is one whole pass of the path over the tall workload
(4,194,304 x 32 FP32, s = 256, r1 = 2048, r2 = 16, s_out = 8000): the FCT1
sketch (pass 1), the FP64 QR, the row-norm pass (pass 2), the Bernoulli
selection, the gather and the FP64 coreset solve, all through l1_regress.
Inputs are resident in HBM before the timed region.

value = algorithmic bytes of the two streaming passes (X read twice, lambda
written once) per step / step time.  The dominant kernel's roofline entry
uses the pass-1 kernel's own device time, measured with HIP events around its
launches on the stream it runs on; its HBM traffic comes from the committed
counter summary when that summary was taken on the current kernel source.
The CPU oracle runs the whole path (steps 1-8) once on the same workload on
one host core.  --workload precision|large times the same steps on the
33,554,432 x 64 or 268,435,456 x 16 workloads.  The batching workload (256 instances of uneven n and d) is
timed as one batch against the same instances solved one after another.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Π1A + sampling pass GB/s (% HBM peak); ℓ1 solve time at (1+ε) opt, plain vs BF16"
HBM_PEAK_GBS = 8000.0


def cpu_oracle_run(A, b, w, rows: int):
    """Time the oracle's whole path (steps 1-8) on the first `rows` rows, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import pipeline
    rows = min(rows, w.n)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        out = pipeline.l1_regress(A[:, :rows].T, b[:rows], s=w.s, r1=w.r1, r2=w.r2,
                                  s_out=w.s_out, seed=w.seed)
        dt = time.perf_counter() - t0
    q = w.d + 1
    nbytes = 2 * rows * q * 4 + rows * 4
    return dict(value=nbytes / dt / 1e9, unit="GB/s", cores=1, kind="oracle",
                sample=f"{rows} of {w.n} rows, steps 1-8 (sketch, QR, row norms, selection, "
                       f"coreset LP of {out['idx'].size} rows), {dt:.2f} s")


def committed_traffic(kernel_sources_sha: str, path: str):
    """HBM bytes per pass-1 launch from the committed counter summary, or None
    if it is missing or was taken on other kernel source."""
    try:
        with open(path) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines() if ": " in line)
    except OSError:
        return None
    if kv.get("source_sha256", "").strip() != kernel_sources_sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_copy_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Read + write bandwidth of a device-to-device copy of `mib` MiB (torch's
    copy on its current stream, timed with events on that stream): the
    streaming bandwidth this machine reaches, beside the nominal HBM peak."""
    src = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def bench_batched(F, ctx, count: int, steps: int, progress):
    """The batching workload: `count` instances of uneven n and d solved in one
    batch (captured graph, block size s autotuned per d), against the same
    instances solved one after another by the single-instance path with the
    block sizes the tuner chose."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import synth
    ws = synth.batch_instances(count)
    items = []
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        for k, (w, (A, b, _)) in enumerate(zip(ws, ex.map(lambda w: synth.generate(w, threads=1), ws))):
            prm = F.params(s=0, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
            items.append(dict(A=torch.from_numpy(A).cuda(), b=torch.from_numpy(b).cuda(),
                              prm=prm, w=w))
            if (k + 1) % 64 == 0:
                progress(f"batch: generated and uploaded {k + 1} of {count} instances")
    torch.cuda.synchronize()
    rows = sum(w.n for w in ws)
    nbytes = sum(2 * w.n * (w.d + 1) * 4 + w.n * 4 for w in ws)
    t0 = time.perf_counter()
    res, st = F.l1_regress_batched(ctx, items, eps=0.05)   # autotunes s and captures the graph
    t_first = time.perf_counter() - t0
    if st != 0:
        bad = [(it["w"].seed, it["w"].n, it["w"].d, r["s"], r["status"])
               for it, r in zip(items, res) if r["status"] != 0]
        raise SystemExit(f"batched solve failed: status {st}; (seed, n, d, s, status): {bad}")
    progress(f"batch: first call (autotune + capture + run) {t_first:.2f} s")
    t0 = time.perf_counter()
    for _ in range(steps):
        res, st = F.l1_regress_batched(ctx, items, eps=0.05)
    torch.cuda.synchronize()
    dt_batch = (time.perf_counter() - t0) / steps
    progress(f"batch: {steps} timed replays, {dt_batch * 1e3:.2f} ms per batch")
    seq_prm = [F.params(s=r["s"], r1=it["w"].r1, r2=it["w"].r2, s_out=it["w"].s_out,
                        seed=it["w"].seed) for it, r in zip(items, res)]
    for it, prm in zip(items, seq_prm):            # warm-up pass
        F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq = [F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05) for it, prm in zip(items, seq_prm)]
    torch.cuda.synchronize()
    dt_seq = (time.perf_counter() - t0) / steps
    progress(f"batch: sequential single-instance path {dt_seq * 1e3:.2f} ms per batch")
    same_S = all(r["S"] == S1 for r, (_, _, S1) in zip(res, seq))
    dev = 0.0
    for it, r, (x1, _, _) in zip(items, res, seq):
        fb = F.fct_l1_objective(ctx, it["A"], it["b"], r["x"])
        f1 = F.fct_l1_objective(ctx, it["A"], it["b"], x1)
        dev = max(dev, abs(fb / f1 - 1))
    ratios = []
    for it, r in list(zip(items, res))[:: max(1, count // 16)]:
        n = it["w"].n
        x_ref, _ = F.l1_solve(ctx, it["A"], it["b"],
                              torch.ones(n, dtype=torch.float64, device="cuda"), iters=120)
        ratios.append(F.fct_l1_objective(ctx, it["A"], it["b"], r["x"]) /
                      F.fct_l1_objective(ctx, it["A"], it["b"], x_ref))
    tuned = {}
    for it, r in zip(items, res):
        tuned[str(it["w"].d)] = r["s"]
    del items
    torch.cuda.empty_cache()
    return {
        "workload": f"batch-{count}: n ~ U[2^14, 2^20], d in {{8,16,32,64}}, f32, "
                    "r1 = 8 d ceil(log2 d), r2 = 16, s_out = 250 (d+1), eps = 0.05",
        "instances": count, "rows": rows, "algorithmic_bytes": nbytes,
        "batched_ms": round(dt_batch * 1e3, 3), "sequential_ms": round(dt_seq * 1e3, 3),
        "speedup": round(dt_seq / dt_batch, 3),
        "batched_rows_per_s": round(rows / dt_batch), "sequential_rows_per_s": round(rows / dt_seq),
        "batched_GBps": round(nbytes / dt_batch / 1e9, 1),
        "batched_hbm_frac": round(nbytes / dt_batch / 1e9 / HBM_PEAK_GBS, 4),
        "first_call_s": round(t_first, 3), "autotuned_s_by_d": tuned,
        "same_coreset_sizes": same_S, "max_objective_deviation_batched_vs_single": dev,
        "objective_ratio_vs_all_rows_solve_max": max(ratios),
        "objective_ratio_sample": f"{len(ratios)} of {count} instances",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=1 << 22)
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device to device (counter scale)")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-ref", action="store_true", help="skip the all-rows reference solve")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batching workload (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--workload", default="tall", choices=("tall", "precision", "large"),
                    help="workload of the timed steps (the bench line is quoted on tall)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design (row shards, one all-reduce of the r1 x q sketch) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1207_4684_amd import fctl1 as F

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    w = {"tall": synth.TALL, "precision": synth.PRECISION, "large": synth.LARGE}[args.workload]
    q = w.d + 1
    A, b, _ = synth.generate(w)
    progress(f"generated {w.name}")
    Ad = torch.from_numpy(A).cuda()
    bd = torch.from_numpy(b).cuda()
    ctx = F.Context(0)
    Al = F.fct_to_bf16(ctx, Ad)
    bl = F.fct_to_bf16(ctx, bd)
    torch.cuda.synchronize()
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)

    def step(lowp: bool):
        if lowp:
            return F.l1_regress(ctx, Ad, bd, prm, eps=w.eps, A_lowp=Al, b_lowp=bl)
        return F.l1_regress(ctx, Ad, bd, prm, eps=w.eps)

    def timed(lowp: bool, steps: int):
        for _ in range(args.warmup):
            step(lowp)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step(lowp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        prof = [ctx.profile_read(k) for k in range(3)]
        ctx.profile(False)
        return dt, prof, out

    dt_plain, prof_plain, (x_plain, _, S_plain) = timed(False, args.steps)
    progress(f"timed {args.steps} plain steps: {dt_plain * 1e3:.3f} ms/step")
    dt_bf16, prof_bf16, (x_bf16, _, S_bf16) = timed(True, args.steps)
    progress(f"timed {args.steps} bf16 steps: {dt_bf16 * 1e3:.3f} ms/step")

    pass1_bytes = w.n * q * 4
    pass2_bytes = w.n * q * 4 + w.n * 4
    pass2_bytes_bf16 = w.n * q * 2 + w.n * 4
    p1_ms = prof_plain[0][0] / max(1, prof_plain[0][1])
    p2_ms = prof_plain[1][0] / max(1, prof_plain[1][1])
    p2b_ms = prof_bf16[1][0] / max(1, prof_bf16[1][1])
    solve_ms = prof_plain[2][0] / max(1, prof_plain[2][1])
    p1_gbs = pass1_bytes / (p1_ms * 1e-3) / 1e9
    value = (pass1_bytes + pass2_bytes) / dt_plain / 1e9

    f_plain = F.fct_l1_objective(ctx, Ad, bd, x_plain)
    f_bf16 = F.fct_l1_objective(ctx, Ad, bd, x_bf16)
    ref = None
    if not args.skip_ref:
        x_ref, _ = F.l1_solve(ctx, Ad, bd, torch.ones(w.n, dtype=torch.float64, device="cuda"),
                              iters=120)
        ref = F.fct_l1_objective(ctx, Ad, bd, x_ref)

    if args.profile_copy_mib > 0:
        src = torch.empty(args.profile_copy_mib << 18, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    from paper_1207_4684_amd.profile_summary import source_sha256
    wave_form = w.s <= 2048  # FP32 data: the wave-level sketch kernel, else the workgroup tile
    p1_kernel = ("pass1_wave_kernel" if w.s <= 256 else "pass1_block_kernel") if wave_form \
        else "pass1_kernel"
    traffic = None
    if wave_form:
        traffic = committed_traffic(source_sha256(), os.path.join(
            ROOT, "profiles", f"pmc_pass1_wave_kernel_{w.name}.txt"))

    copy_gbps = measured_copy_gbps(torch)
    progress(f"device copy: {copy_gbps:.0f} GB/s (read + write)")

    batched = None
    if args.batch > 0:
        batched = bench_batched(F, ctx, args.batch, args.batch_steps, progress)

    if not args.skip_cpu:
        progress("timing the CPU oracle")
    cpu = None if args.skip_cpu else cpu_oracle_run(A, b, w, args.cpu_rows)

    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt_plain * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "s": w.s, "r1": w.r1, "r2": w.r2,
                   "s_out": w.s_out, "eps": w.eps, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(p1_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(p1_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": f"{p1_kernel} (FCT1 sketch, with its random-table kernel)"
                     if wave_form else f"{p1_kernel} (FCT1 sketch)", "kernel_ms": round(p1_ms, 5),
                     "algorithmic_bytes": pass1_bytes,
                     "measured_copy_GBps": round(copy_gbps, 1),
                     "frac_of_measured_copy": round(p1_gbs / copy_gbps, 4)},
        "cpu_baseline": cpu,
        "passes": {
            "pass1_ms": round(p1_ms, 5), "pass1_GBps": round(p1_gbs, 1),
            "pass2_f32_ms": round(p2_ms, 5),
            "pass2_f32_GBps": round(pass2_bytes / (p2_ms * 1e-3) / 1e9, 1),
            "pass2_bf16_ms": round(p2b_ms, 5),
            "pass2_bf16_GBps": round(pass2_bytes_bf16 / (p2b_ms * 1e-3) / 1e9, 1),
            "solve_ms": round(solve_ms, 4),
        },
        "batched": batched,
        "end_to_end": {
            "plain_ms": round(dt_plain * 1e3, 4), "bf16_ms": round(dt_bf16 * 1e3, 4),
            "plain_rows_per_s": round(w.n / dt_plain), "bf16_rows_per_s": round(w.n / dt_bf16),
            "coreset_rows_plain": S_plain, "coreset_rows_bf16": S_bf16,
            "objective_plain": f_plain, "objective_bf16": f_bf16,
            "objective_all_rows_solve": ref,
            "ratio_plain": (f_plain / ref) if ref else None,
            "ratio_bf16": (f_bf16 / ref) if ref else None,
        },
    }
    ctx.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
