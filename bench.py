"""Benchmark of the FastCauchyRegression hot path on one MI355X.

A step is one whole pass of the path over the large workload
(268,435,456 x 16 FP32 with b, s = 1024, r1 = 1024, r2 = 16, s_out = 10000,
eps = 0.01): the FCT1 sketch (pass 1), the FP64 QR, the row-norm pass
(pass 2), the Bernoulli selection, the gather and the FP64 coreset solve, all
through l1_regress.  Inputs are resident in HBM before the timed region, and
a 1 GiB buffer is written between steps so that no step starts with its
input in the 256 MB MALL.

value = algorithmic bytes of the two streaming passes (X read twice, lambda
written once) / median step time.  The roofline entry is pass 1's kernel
(the bucket-owner sketch kernel), timed with HIP events around its launches
on the stream it runs on; its HBM traffic comes from the committed counter
summary when that summary was taken on the current kernel source.  The same
line carries pass 2 (FP32 and BF16), the solve, the BF16 path's error against
the library's FP64 pass 2, the precision (33,554,432 x 64), tall
(4,194,304 x 32) and small (65,536 x 16 FP64) workloads, and the batching
workload (256 instances).  The CPU baseline runs the oracle's steps on a
bounded sample of the large workload in worker processes on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Π1A + sampling pass GB/s (% HBM peak); ℓ1 solve time at (1+ε) opt, plain vs BF16"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
# second (one wave64 VALU instruction takes 4 cycles of a 16-lane SIMD)
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# VALU instructions per C entry of the FCT2 contraction's inner loop (the
# 17-column slice compiled for gfx950: 228 per Philox call of 4 entries, 68 of
# them FP64 FMAs): 40 to draw and transform the variate plus one FMA per column
FCT2_GEN_VALU_PER_ENTRY = 40
CHUNK = 1 << 20


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- CPU baseline: the oracle on the host's cores ----------------------------

def _cpu_worker(conn, wname, chunks):
    """One worker of the CPU baseline: generates its chunks of the workload
    (not timed), then runs the oracle's per-row stages on command."""
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import synth
    from oracle import basis, fct, philox, sampling
    w = getattr(synth, wname)
    q = w.d + 1
    cctx = synth.chunk_context(w)
    data = []
    for c in chunks:
        A, b = synth.generate_chunk(w, c, cctx)
        data.append((c * CHUNK, np.hstack([A.T.astype(np.float64), -b.astype(np.float64)[:, None]])))
    conn.send("ready")
    lams = []
    while True:
        cmd, arg = conn.recv()
        if cmd == "sketch":
            t0 = time.perf_counter()
            Y = np.zeros((w.r1, q))
            for row0, X in data:
                Y += fct.pi1_apply(X, w.s, w.r1, w.seed, row0=row0)
            conn.send((Y, time.perf_counter() - t0))
        elif cmd == "lambda":
            R = arg
            t0 = time.perf_counter()
            M = basis.m_matrix(R, w.seed, w.r2)
            lams = [sampling.row_norm_estimates(X, M) for _, X in data]
            conn.send((float(sum(l.sum() for l in lams)), time.perf_counter() - t0))
        elif cmd == "select":
            s_out, total = arg
            t0 = time.perf_counter()
            rows, wts = [], []
            for (row0, X), lam in zip(data, lams):
                p = sampling.probabilities(lam, s_out, total)
                words = philox.sample_words(w.seed, X.shape[0], start=row0).astype(np.uint64)
                keep = np.nonzero(words < sampling.thresholds(p))[0]
                rows.append(X[keep])
                wts.append(1.0 / p[keep])
            conn.send((np.vstack(rows), np.concatenate(wts), time.perf_counter() - t0))
        else:
            conn.close()
            return


def cpu_baseline(wname: str, sample_rows: int):
    """The oracle's steps 1-8 on the first sample_rows rows of workload wname:
    sketch, row norms and selection in P worker processes (P = the host cores
    this process may use, one thread each), QR, M and the coreset LP in this
    process.  Returns the record and per-stage seconds."""
    import multiprocessing as mp
    import synth
    from oracle import basis, l1
    w = getattr(synth, wname)
    P = len(os.sched_getaffinity(0))
    nch = max(1, sample_rows // CHUNK)
    P = min(P, nch)
    plan = [list(range(i, nch, P)) for i in range(P)]
    ctx = mp.get_context("spawn")
    conns, procs = [], []
    for i in range(P):
        a, b = ctx.Pipe()
        pr = ctx.Process(target=_cpu_worker, args=(b, wname, plan[i]), daemon=True)
        pr.start()
        conns.append(a)
        procs.append(pr)
    for c in conns:
        assert c.recv() == "ready"
    stages = {}
    t_all = time.perf_counter()
    for c in conns:
        c.send(("sketch", None))
    outs = [c.recv() for c in conns]
    Y = sum(o[0] for o in outs)
    stages["pass1_sketch"] = max(o[1] for o in outs)
    t0 = time.perf_counter()
    R = basis.qr_r(Y)
    stages["qr"] = time.perf_counter() - t0
    for c in conns:
        c.send(("lambda", R))
    outs = [c.recv() for c in conns]
    total = sum(o[0] for o in outs)
    stages["pass2_row_norms"] = max(o[1] for o in outs)
    for c in conns:
        c.send(("select", (w.s_out, total)))
    outs = [c.recv() for c in conns]
    stages["selection"] = max(o[2] for o in outs)
    Xs = np.vstack([o[0] for o in outs])
    ws = np.concatenate([o[1] for o in outs])
    t0 = time.perf_counter()
    x, _ = l1.lp(Xs[:, :-1], -Xs[:, -1], ws)
    stages["coreset_lp"] = time.perf_counter() - t0
    wall = time.perf_counter() - t_all
    for c in conns:
        c.send(("stop", None))
    for pr in procs:
        pr.join(timeout=30)
    rows = nch * CHUNK
    q = w.d + 1
    nbytes = 2 * rows * q * 4 + rows * 4
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    stage_sum = sum(stages.values())
    return {"value": round(nbytes / stage_sum / 1e9, 4), "unit": "GB/s", "cores": P, "kind": "oracle",
            "sample": f"first {rows} of {w.n} rows of {w.name}, steps 1-8 (sketch, QR, row norms, "
                      f"selection, coreset LP of {Xs.shape[0]} rows), stage times summed "
                      f"(the per-row stages run on {P} worker processes, one thread each)",
            "cpu_model": model, "stages_s": {k: round(v, 3) for k, v in stages.items()},
            "wall_s": round(wall, 3)}


# ---- GPU timing helpers -------------------------------------------------------

class Flusher:
    """A 1 GiB buffer written between timed steps (evicts the MALL)."""

    def __init__(self, torch):
        self.buf = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        self.torch = torch

    def __call__(self):
        self.buf.fill_(1.0)


def timed_steps(torch, step, steps: int, warmup: int, flush):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times, out = [], None
    for _ in range(steps):
        flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times, out


def measured_copy_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Read + write bandwidth of a device-to-device copy of `mib` MiB (torch's
    copy on its current stream, timed with events on that stream)."""
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


def jaccard(a, b):
    a, b = set(a.tolist()), set(b.tolist())
    return len(a & b) / max(1, len(a | b))


def run_workload(F, torch, ctx, w, steps, warmup, flush, bf16=True, ref=True, err_report=False,
                 multi=0, fct2=None):
    """Time l1_regress on workload w (plain and, for FP32 data, the BF16
    sampling pass); pass times from the library's events; objectives from the
    library (fct_l1_objective) against an all-rows solve by the library."""
    import synth
    t0 = time.perf_counter()
    A, b, _ = synth.generate(w, threads=min(16, len(os.sched_getaffinity(0))))
    progress(f"{w.name}: generated in {time.perf_counter() - t0:.1f} s")
    Ad = torch.from_numpy(A).cuda()
    bd = torch.from_numpy(b).cuda()
    del A, b
    f64 = w.dtype == "f64"
    q = w.d + 1
    es = 8 if f64 else 4
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    rec = {"workload": w.name, "n": w.n, "d": w.d, "s": w.s, "r1": w.r1, "r2": w.r2,
           "s_out": w.s_out, "eps": w.eps, "dtype": w.dtype}
    pass1_bytes = w.n * q * es
    pass2_bytes = w.n * q * es + w.n * 4
    pass2_bytes_bf16 = w.n * q * 2 + w.n * 4

    def time_path(lowp, Al=None, bl=None):
        def step():
            if lowp:
                return F.l1_regress(ctx, Ad, bd, prm, eps=w.eps, A_lowp=Al, b_lowp=bl)
            return F.l1_regress(ctx, Ad, bd, prm, eps=w.eps)
        ctx.profile(False)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ctx.profile(True)
        times, out = timed_steps(torch, step, steps, 0, flush)
        prof = [ctx.profile_read(k) for k in range(3)]
        ctx.profile(False)
        return times, prof, out

    t_plain, prof_plain, (x_plain, _, S_plain) = time_path(False)
    med = statistics.median(t_plain)
    progress(f"{w.name}: {steps} plain steps, median {med * 1e3:.3f} ms")
    p1_ms = prof_plain[0][0] / max(1, prof_plain[0][1])
    p2_ms = prof_plain[1][0] / max(1, prof_plain[1][1])
    solve_ms = prof_plain[2][0] / max(1, prof_plain[2][1])
    rec.update({
        "plain_ms": round(med * 1e3, 4), "plain_mean_ms": round(statistics.mean(t_plain) * 1e3, 4),
        "plain_rows_per_s": round(w.n / med), "GBps_two_passes": round((pass1_bytes + pass2_bytes) / med / 1e9, 1),
        "pass1_ms": round(p1_ms, 5), "pass1_GBps": round(pass1_bytes / (p1_ms * 1e-3) / 1e9, 1),
        "pass1_frac": round(pass1_bytes / (p1_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "pass2_ms": round(p2_ms, 5), "pass2_GBps": round(pass2_bytes / (p2_ms * 1e-3) / 1e9, 1),
        "pass2_frac": round(pass2_bytes / (p2_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "solve_ms": round(solve_ms, 4), "coreset_rows_plain": S_plain,
    })
    # determinism: the same call again gives the same bits
    x_again, _, S_again = F.l1_regress(ctx, Ad, bd, prm, eps=w.eps)
    rec["rerun_bitwise_equal"] = bool(S_again == S_plain and np.array_equal(x_again, x_plain))
    f_plain = F.fct_l1_objective(ctx, Ad, bd, x_plain)
    rec["objective_plain"] = f_plain
    if bf16 and not f64:
        Al, bl = F.fct_to_bf16(ctx, Ad), F.fct_to_bf16(ctx, bd)
        t_bf, prof_bf, (x_bf, _, S_bf) = time_path(True, Al, bl)
        medb = statistics.median(t_bf)
        p2b_ms = prof_bf[1][0] / max(1, prof_bf[1][1])
        rec.update({
            "bf16_ms": round(medb * 1e3, 4), "bf16_rows_per_s": round(w.n / medb),
            "pass2_bf16_ms": round(p2b_ms, 5),
            "pass2_bf16_GBps": round(pass2_bytes_bf16 / (p2b_ms * 1e-3) / 1e9, 1),
            "pass2_bf16_frac": round(pass2_bytes_bf16 / (p2b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "coreset_rows_bf16": S_bf, "objective_bf16": F.fct_l1_objective(ctx, Ad, bd, x_bf),
            "bf16_copy_ms": None,
        })
        progress(f"{w.name}: {steps} bf16 steps, median {medb * 1e3:.3f} ms")
        # the BF16 copy's own cost (both accountings: a copy made per solve
        # adds it to the BF16 path)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            F.fct_to_bf16(ctx, Ad)
            F.fct_to_bf16(ctx, bd)
        torch.cuda.synchronize()
        rec["bf16_copy_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 4)
        if err_report:
            rec["bf16_error"] = bf16_error_report(F, torch, ctx, w, Ad, bd, Al, bl)
        del Al, bl
    xs_multi = {}
    if multi > 0 and not f64:
        # K coresets (and solves) from one sampling pass, both kinds of draw
        m = {"K": multi, "single_plain_ms": rec["plain_ms"]}
        for name, mode in (("bernoulli", F.FCT_SAMPLE_BERNOULLI), ("replace", F.FCT_SAMPLE_REPLACE)):
            def mstep():
                return F.l1_regress_multi(ctx, Ad, bd, prm, multi, mode, eps=w.eps)
            t_m, out_m = timed_steps(torch, mstep, 3, 1, flush)
            tm = statistics.median(t_m)
            xs_multi[name] = out_m[0]
            m[f"{name}_ms"] = round(tm * 1e3, 4)
            m[f"{name}_solutions_per_s"] = round(multi / tm, 1)
            m[f"{name}_speedup_vs_single_calls"] = round(multi * med / tm, 3)
            m[f"{name}_coreset_rows"] = [int(v) for v in out_m[2]]
        rec["multi"] = m
        progress(f"{w.name}: {multi} draws per pass: bernoulli {m['bernoulli_ms']} ms, "
                 f"replace {m['replace_ms']} ms")
    x_fct2 = None
    if fct2 is not None and not f64:
        rec["fct2"], x_fct2 = bench_fct2(F, torch, ctx, w, Ad, bd, flush, **fct2)
    if ref:
        x_ref, _ = F.l1_solve(ctx, Ad, bd, torch.ones(w.n, dtype=torch.float64, device="cuda"),
                              iters=120)
        f_ref = F.fct_l1_objective(ctx, Ad, bd, x_ref)
        rec["objective_all_rows_solve"] = f_ref
        rec["ratio_plain"] = f_plain / f_ref
        if "objective_bf16" in rec:
            rec["ratio_bf16"] = rec["objective_bf16"] / f_ref
        for name, X in xs_multi.items():
            rec["multi"][f"{name}_ratio_max"] = max(
                F.fct_l1_objective(ctx, Ad, bd, X[k]) / f_ref for k in range(X.shape[0]))
        if x_fct2 is not None:
            rec["fct2"]["regress_ratio"] = F.fct_l1_objective(ctx, Ad, bd, x_fct2) / f_ref
    del Ad, bd
    torch.cuda.empty_cache()
    return rec


def bench_fct2(F, torch, ctx, w, Ad, bd, flush, t=4096, s=32, steps=5, overlap=False):
    """The FCT2 sketch Pi1 [A, -b] (block size t, s sampled rows per block,
    r1 of the workload) and the regression that takes its R from it.  Kernel
    times from the library's events: the FJLT blocks read X once and write
    G z (HBM); the contraction generates r1 x (n s / t) Cauchy variates
    (VALU)."""
    q = w.d + 1
    nb = -(-w.n // t)
    K = nb * s
    qc = 8 if q <= 8 else 17 if q <= 17 else 33
    zq = -(-q // qc) * qc
    valu_per_entry = (zq // qc) * FCT2_GEN_VALU_PER_ENTRY + zq
    def sketch():
        return F.fct2_sketch(ctx, Ad, bd, t, s, w.r1, w.seed, want_y=False)
    # the default launch (each kernel alone on the device: per-kernel
    # rooflines); with ``overlap`` also the option that runs the contraction
    # of one segment beside the FJLT of the next
    ctx.profile(True)
    times, _ = timed_steps(torch, sketch, steps, 1, flush)
    fj = ctx.profile_read(3)
    ca = ctx.profile_read(4)
    ctx.profile(False)
    t_ov = None
    if overlap:
        ctx.set_option(F.FCT_OPT_FCT2_OVERLAP, 1)
        t_ov, _ = timed_steps(torch, sketch, steps, 1, flush)
        ctx.set_option(F.FCT_OPT_FCT2_OVERLAP, 0)
    fj_ms = fj[0] / max(1, fj[1])
    ca_ms = ca[0] / max(1, ca[1])
    fj_bytes = w.n * q * 4 + K * zq * 8
    entries = w.r1 * K
    out = {"t": t, "s": s, "r1": w.r1, "sketch_ms": round(statistics.median(times) * 1e3, 4),
           "sketch_overlap_option_ms": None if t_ov is None else round(statistics.median(t_ov) * 1e3, 4),
           "fjlt_ms": round(fj_ms, 5), "fjlt_algorithmic_bytes": fj_bytes,
           "fjlt_GBps": round(fj_bytes / (fj_ms * 1e-3) / 1e9, 1),
           "fjlt_frac": round(fj_bytes / (fj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "contraction_ms": round(ca_ms, 5), "cauchy_entries": entries,
           "cauchy_entries_per_s": round(entries / (ca_ms * 1e-3)),
           "contraction_valu_lane_ops_per_entry": valu_per_entry,
           "contraction_valu_frac": round(entries * valu_per_entry / (ca_ms * 1e-3) / VALU_PEAK_LANE_OPS, 4)}
    prm = F.params(s=t, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed, flags=F.FCT_FLAG_FCT2, s2=s)
    tr, res = timed_steps(torch, lambda: F.l1_regress(ctx, Ad, bd, prm, eps=w.eps), 3, 1, flush)
    out.update({"regress_ms": round(statistics.median(tr) * 1e3, 4), "regress_coreset_rows": int(res[2])})
    from paper_1207_4684_amd.profile_summary import FCT2_SOURCES, source_sha256
    tr_b = committed_traffic(source_sha256(FCT2_SOURCES), os.path.join(
        ROOT, "profiles", f"pmc_fct2_fjlt_{w.name}.txt"))
    out["fjlt_traffic"] = None if tr_b is None or (t, s) != (4096, 32) else round(tr_b)
    progress(f"{w.name}: FCT2 sketch {out['sketch_ms']} ms (FJLT {out['fjlt_ms']} ms, "
             f"contraction {out['contraction_ms']} ms), regression {out['regress_ms']} ms")
    return out, res[0]


def bf16_error_report(F, torch, ctx, w, Ad, bd, Al, bl):
    """The BF16 sampling pass against the library's FP64 pass 2 on the same R
    (X promoted to FP64 on the device): the distribution of lambda_bf16 /
    lambda_64, the largest relative error of p, and the overlap of the
    selected rows with the FP32 and FP64 selections (same seed); for the
    plain form [A_bf16, -b_bf16] with R and for the residual form
    [A_bf16, -r0_bf16] with R T (fct_lowp_residual)."""
    _, R = F.fct_sketch(ctx, Ad, bd, w.s, w.r1, w.seed, want_y=False)
    lam32, p32, t32 = F.l1_sample_probs(ctx, Ad, bd, R, w.r2, w.seed, w.s_out)
    A64, b64 = Ad.double(), bd.double()
    lam64, p64, t64 = F.l1_sample_probs(ctx, A64, b64, R, w.r2, w.seed, w.s_out)
    del A64, b64
    torch.cuda.empty_cache()
    cap = 4 * w.s_out + 1024
    i32 = F.l1_select(ctx, lam32, t32, w.s_out, w.seed, cap)[0].cpu().numpy()
    i64 = F.l1_select(ctx, lam64, t64, w.s_out, w.seed, cap)[0].cpu().numpy()

    def figures(lamb, pb, tb):
        ratio = (lamb.double() / lam64.double())[lam64 > 0]
        qs = torch.quantile(ratio[:: max(1, ratio.numel() // (1 << 24))],
                            torch.tensor([0.01, 0.5, 0.99], dtype=torch.float64, device="cuda"))
        inside = ((ratio >= 0.5) & (ratio <= 1.5)).double().mean()
        pm = p64.double() > 0
        prel = ((pb.double() - p64.double()).abs() / p64.double())[pm].max()
        ib = F.l1_select(ctx, lamb, tb, w.s_out, w.seed, cap)[0].cpu().numpy()
        return {"lambda_ratio_p01_p50_p99": [round(float(v), 5) for v in qs.tolist()],
                "lambda_ratio_frac_in_half_to_three_halves": round(float(inside), 6),
                "p_max_rel_err": float(prel),
                "sum_lambda_rel_err": float(abs(tb.item() / t64.item() - 1)),
                "jaccard_idx_bf16_vs_f32": round(jaccard(ib, i32), 5),
                "jaccard_idx_bf16_vs_f64": round(jaccard(ib, i64), 5)}

    out = {"reference": "library FP64 pass 2 (FP64 data and M) on the same R"}
    out.update(figures(*F.l1_sample_probs(ctx, Al, bl, R, w.r2, w.seed, w.s_out)))
    out["jaccard_idx_f32_vs_f64"] = round(jaccard(i32, i64), 5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r_lowp, Rres = F.fct_lowp_residual(ctx, Ad, bd, R)
    e1.record()
    torch.cuda.synchronize()
    res = figures(*F.l1_sample_probs(ctx, Al, r_lowp, Rres, w.r2, w.seed, w.s_out))
    res["residual_column_ms"] = round(e0.elapsed_time(e1), 4)
    out["residual_form"] = res
    return out


def bench_mrhs_subspace(F, torch, ctx, flush, k: int = 8):
    """Multiple l1 regression with k right-hand sides and l1 subspace
    approximation on the tall generator (4,194,304 rows): one sketch and
    sampling pass for all the regressions against k (or d) single ones."""
    import synth
    w = synth.TALL
    A, b, _ = synth.generate(w, threads=min(16, len(os.sched_getaffinity(0))))
    Ad, bd = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
    rng = np.random.default_rng(1)
    # k right-hand sides: b, and planted fits A x_j with Laplace noise and 2%
    # Cauchy outliers
    Bh = np.empty((k, w.n), dtype=np.float32)
    Bh[0] = b
    xs = rng.standard_normal((w.d, k - 1))
    Bh[1:] = (A.T.astype(np.float64) @ xs).T + rng.laplace(0, 0.1, (k - 1, w.n))
    out_rows = rng.choice(w.n, w.n // 50, replace=False)
    Bh[1:, out_rows] = 1e3 * rng.standard_cauchy((k - 1, out_rows.size))
    Bd = torch.from_numpy(Bh).cuda()
    del A, b, Bh
    q = w.d + k
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    out = {"workload": f"{w.name}, {k} right-hand sides", "k": k}
    t_m, res = timed_steps(torch, lambda: F.l1_regress_mrhs(ctx, Ad, Bd, prm, eps=w.eps), 3, 1, flush)
    t_s, _ = timed_steps(torch, lambda: [F.l1_regress(ctx, Ad, Bd[j], prm, eps=w.eps) for j in range(k)],
                         3, 1, flush)
    out.update({"mrhs_ms": round(statistics.median(t_m) * 1e3, 4),
                "single_calls_ms": round(statistics.median(t_s) * 1e3, 4),
                "speedup": round(statistics.median(t_s) / statistics.median(t_m), 3),
                "coreset_rows": int(res[2]),
                "algorithmic_GBps": round(2 * w.n * (w.d + k) * 4 / statistics.median(t_m) / 1e9, 1)})
    # subspace approximation of the points [A, b] (d + 1 = 33 coordinates)
    X = torch.cat([Ad, bd[None, :]], dim=0).contiguous()
    prs = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    t_p, rp = timed_steps(torch, lambda: F.l1_subspace(ctx, X, prs, eps=w.eps), 3, 1, flush)
    out.update({"subspace_points": f"{w.n} x {w.d + 1}", "subspace_ms": round(statistics.median(t_p) * 1e3, 4),
                "subspace_j_star": int(rp[2]), "subspace_coreset_rows": int(rp[3])})
    del Ad, bd, Bd, X
    torch.cuda.empty_cache()
    return out


def bench_batched(F, ctx, count: int, steps: int):
    """The batching workload: `count` instances of uneven n and d solved in one
    batch (captured graph, block size s from the library's rule per d), against the same
    instances solved one after another by the single-instance path with the
    block sizes the tuner chose."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import synth
    ws = synth.batch_instances(count)
    items = []
    with ThreadPoolExecutor(max_workers=16) as ex:
        for k, (w, (A, b, _)) in enumerate(zip(ws, ex.map(lambda w: synth.generate(w, threads=1), ws))):
            prm = F.params(s=0, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
            items.append(dict(A=torch.from_numpy(A).cuda(), b=torch.from_numpy(b).cuda(),
                              prm=prm, w=w))
    torch.cuda.synchronize()
    progress(f"batch: generated and uploaded {count} instances")
    rows = sum(w.n for w in ws)
    nbytes = sum(2 * w.n * (w.d + 1) * 4 + w.n * 4 for w in ws)
    t0 = time.perf_counter()
    res, st = F.l1_regress_batched(ctx, items, eps=0.05)   # chooses s and captures the graph
    t_first = time.perf_counter() - t0
    if st != 0:
        bad = [(it["w"].seed, it["w"].n, it["w"].d, r["s"], r["status"])
               for it, r in zip(items, res) if r["status"] != 0]
        raise SystemExit(f"batched solve failed: status {st}; (seed, n, d, s, status): {bad}")
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, st = F.l1_regress_batched(ctx, items, eps=0.05)
        times.append(time.perf_counter() - t0)
    dt_batch = statistics.median(times)
    progress(f"batch: {steps} timed replays, median {dt_batch * 1e3:.2f} ms per batch")
    seq_prm = [F.params(s=r["s"], r1=it["w"].r1, r2=it["w"].r2, s_out=it["w"].s_out,
                        seed=it["w"].seed) for it, r in zip(items, res)]
    for it, prm in zip(items, seq_prm):            # warm-up pass
        F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05) for it, prm in zip(items, seq_prm)]
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    same_S = all(r["S"] == S1 for r, (_, _, S1) in zip(res, seq))
    dev = 0.0
    for it, r, (x1, _, _) in zip(items, res, seq):
        fb = F.fct_l1_objective(ctx, it["A"], it["b"], r["x"])
        f1 = F.fct_l1_objective(ctx, it["A"], it["b"], x1)
        dev = max(dev, abs(fb / f1 - 1))
    tuned = {str(it["w"].d): r["s"] for it, r in zip(items, res)}
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
        "first_call_s": round(t_first, 3), "block_size_by_d": tuned,
        "same_coreset_sizes": same_S, "max_objective_deviation_batched_vs_single": dev,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=("large", "precision", "tall", "small"),
                    help="workload of the headline line (default: the large workload)")
    ap.add_argument("--extras", default="precision,tall,small",
                    help="other workloads timed into the line (comma list; '' = none)")
    ap.add_argument("--extra-steps", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256, help="instances of the batching workload (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-mrhs", dest="mrhs", action="store_false",
                    help="skip the multiple-regression and subspace timings")
    ap.add_argument("--multi", type=int, default=16,
                    help="coresets per sampling pass timed on the headline workload (0 = skip)")
    ap.add_argument("--fct2-t", type=int, default=4096,
                    help="FCT2 block size timed on the headline workload (0 = skip)")
    ap.add_argument("--fct2-s", type=int, default=32, help="FCT2 rows sampled per block")
    ap.add_argument("--fct2-overlap", action="store_true",
                    help="also time FCT2 with FCT_OPT_FCT2_OVERLAP (segmented, two streams)")
    ap.add_argument("--cpu-rows", type=int, default=1 << 26, help="rows of the CPU baseline's sample")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-ref", action="store_true", help="skip the all-rows reference solves")
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device to device (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design (row shards, one all-reduce of the r1 x q sketch) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1207_4684_amd import fctl1 as F

    names = {"large": synth.LARGE, "precision": synth.PRECISION, "tall": synth.TALL,
             "small": synth.SMALL}
    w = names[args.workload]
    ctx = F.Context(0)
    flush = Flusher(torch)
    head = run_workload(F, torch, ctx, w, args.steps, args.warmup, flush, ref=not args.skip_ref,
                        err_report=w.dtype == "f32", multi=args.multi,
                        fct2=dict(t=args.fct2_t, s=args.fct2_s, overlap=args.fct2_overlap)
                        if args.fct2_t > 0 else None)
    if args.profile_copy_mib > 0:
        src = torch.empty(args.profile_copy_mib << 18, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbps = measured_copy_gbps(torch)
    progress(f"device copy: {copy_gbps:.0f} GB/s (read + write)")

    extras = {}
    for name in [x for x in args.extras.split(",") if x and x != args.workload]:
        extras[name] = run_workload(F, torch, ctx, names[name], args.extra_steps, 2, flush,
                                    ref=not args.skip_ref and name != "precision",
                                    err_report=name == "precision")
    batched = bench_batched(F, ctx, args.batch, args.batch_steps) if args.batch > 0 else None
    mrhs = bench_mrhs_subspace(F, torch, ctx, flush) if args.mrhs else None
    del flush
    ctx.close()
    torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu:
        progress("timing the CPU oracle")
        cpu = cpu_baseline("LARGE" if args.workload == "large" else
                           {"precision": "PRECISION", "tall": "TALL", "small": "SMALL"}[args.workload],
                           min(args.cpu_rows, w.n))
        progress(f"CPU oracle: {cpu['stages_s']} on {cpu['cores']} cores")

    from paper_1207_4684_amd.profile_summary import source_sha256
    q = w.d + 1
    es = 8 if w.dtype == "f64" else 4
    pass1_bytes = w.n * q * es
    owner = w.dtype == "f32" and w.s <= 1024 and w.r1 <= 1024
    kernel = ("pass1_owner_kernel (FCT1 sketch, bucket-owner form)" if owner else
              "pass1_wave_kernel / pass1_block_kernel (FCT1 sketch, with its random-table kernel)"
              if w.dtype == "f32" else "pass1_kernel (FCT1 sketch)")
    traffic = committed_traffic(source_sha256(), os.path.join(
        ROOT, "profiles", f"pmc_pass1_{w.name}.txt"))
    p1_gbs = head["pass1_GBps"]
    med_s = head["plain_ms"] * 1e-3
    rec = {
        "metric": METRIC,
        "value": head["GBps_two_passes"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["plain_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "s": w.s, "r1": w.r1, "r2": w.r2,
                   "s_out": w.s_out, "eps": w.eps, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": p1_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(p1_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": kernel, "kernel_ms": head["pass1_ms"],
                     "algorithmic_bytes": pass1_bytes,
                     "measured_copy_GBps": round(copy_gbps, 1),
                     "frac_of_measured_copy": round(p1_gbs / copy_gbps, 4)},
        "cpu_baseline": cpu,
        "timing": "median of the timed steps; a 1 GiB buffer is written before each step",
        "rows_per_s": round(w.n / med_s),
        "end_to_end": head,
        "workloads": extras,
        "batched": batched,
        "multiple_rhs_and_subspace": mrhs,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
