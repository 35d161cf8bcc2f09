"""Text summaries of rocprofv3 result databases (rocpd SQLite files).

    python -m paper_1207_4684_amd.profile_summary stats DB [--match SUBSTR]
    python -m paper_1207_4684_amd.profile_summary traffic FETCH_DB WRITE_DB \
        --kernel SUBSTR --copy-bytes N --algorithmic-bytes B
    python -m paper_1207_4684_amd.profile_summary pmc FETCH_DB WRITE_DB
    python -m paper_1207_4684_amd.profile_summary counters DB [DB ...] --match SUBSTR

``stats`` prints calls, total, average, minimum and maximum device time per
kernel from the kernel trace.  ``traffic`` reads one database collected with
``--pmc FETCH_SIZE`` and one with ``--pmc WRITE_SIZE`` (KiB per dispatch),
scales each by what the same counter reads for the largest dispatch of the
copy kernel (``--copy-kernel``, a copy of ``--copy-bytes`` bytes reads and
writes that many bytes) in the same run, and prints the HBM bytes per launch of the kernels
whose names contain the ``--kernel`` substrings (summed), with the SHA-256 of the sources that build
it so a reader can tell whether the figures still describe the current code.
``counters`` prints the mean per dispatch of every counter in the databases
for the kernels whose names contain ``--match``, and the ratios read from the
shader-sequencer counters when they are present: VALU instructions per wave,
the share of wave time a VALU instruction is issued, LDS bank-conflict cycles
per LDS-busy cycle, and MFMA busy cycles per SQ busy cycle.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PASS1_SOURCES = ("csrc/pass1_owner.hip", "csrc/pass1_wave.hip", "csrc/wave_fwht.h",
                 "csrc/fct_device.h")
FCT2_SOURCES = ("csrc/fct2.hip", "csrc/fct_device.h", "csrc/fct_kernels.h")
SOURCES = {"pass1": PASS1_SOURCES, "fct2": FCT2_SOURCES}


def source_sha256(files=PASS1_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_stats(db: str, match: str | None = None):
    """Per kernel: calls, total ms, mean, min, max, median and the mean over
    all dispatches but the first (the first launch of a kernel in a process
    also pays its one-time set-up; a benchmark's warmup steps absorb it) in us."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, end - start from kernels order by start").fetchall()
    con.close()
    agg: dict[str, list[float]] = {}
    for name, dur in rows:
        if match and match not in name:
            continue
        agg.setdefault(name, []).append(float(dur))
    out = []
    for name, d in agg.items():
        srt = sorted(d)
        med = srt[len(srt) // 2] if len(srt) % 2 else 0.5 * (srt[len(srt) // 2 - 1] + srt[len(srt) // 2])
        rest = d[1:] if len(d) > 1 else d
        out.append((name, len(d), sum(d) / 1e6, sum(d) / len(d) / 1e3, min(d) / 1e3, max(d) / 1e3,
                    med / 1e3, sum(rest) / len(rest) / 1e3))
    out.sort(key=lambda r: -r[2])
    return out


def counter_per_dispatch(db: str, counter: str):
    """(kernel name, mean counter value per dispatch, dispatches) per kernel."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, dispatch_id, sum(value) from counters_collection "
        "where counter_name = ? group by kernel_name, dispatch_id", (counter,)).fetchall()
    con.close()
    agg: dict[str, list[float]] = {}
    for name, _, v in rows:
        agg.setdefault(name, []).append(float(v))
    return {k: (sum(v) / len(v), len(v), max(v)) for k, v in agg.items()}


def _short(name: str, width: int = 90) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def cmd_stats(args):
    print(f"# kernel trace summary of {os.path.basename(args.db)}")
    print(f"{'kernel':90s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
          f"{'median_us':>10s} {'avg_after_first_us':>18s}")
    for name, n, tot, avg, mn, mx, med, avg1 in kernel_stats(args.db, args.match):
        print(f"{_short(name):90s} {n:6d} {tot:10.3f} {avg:10.2f} {mn:10.2f} {mx:10.2f} {med:10.2f} {avg1:18.2f}")


def _copy_value(table, pattern):
    cands = [(mx, v, n, k) for k, (v, n, mx) in table.items() if pattern in k.lower()]
    if not cands:
        raise SystemExit("no copy kernel in the counter database")
    mx, v, n, k = max(cands)
    return mx, k


def cmd_traffic(args):
    fetch = counter_per_dispatch(args.fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(args.write_db, "WRITE_SIZE")
    cf, cf_name = _copy_value(fetch, args.copy_kernel.lower())
    cw, cw_name = _copy_value(write, args.copy_kernel.lower())
    f_scale = args.copy_bytes / (cf * 1024.0)
    w_scale = args.copy_bytes / (cw * 1024.0)
    # one launch of the measured unit is one dispatch of each named kernel
    hbm = 0.0
    for sub in args.kernel:
        fk = [k for k in fetch if sub in k]
        wk = [k for k in write if sub in k]
        if not fk or not wk:
            raise SystemExit(f"kernel {sub!r} not found in the counter databases")
        f_val, f_n, _ = fetch[fk[0]]
        w_val, w_n, _ = write[wk[0]]
        hbm += f_val * 1024.0 * f_scale + w_val * 1024.0 * w_scale
        print(f"kernel: {fk[0]}")
        print(f"dispatches_fetch: {f_n}")
        print(f"dispatches_write: {w_n}")
        print(f"fetch_kib_per_dispatch: {f_val:.1f}")
        print(f"write_kib_per_dispatch: {w_val:.1f}")
    print(f"copy_kernel: {cf_name}")
    print(f"copy_bytes: {args.copy_bytes}")
    print(f"copy_fetch_kib: {cf:.1f}")
    print(f"copy_write_kib: {cw:.1f}")
    print(f"fetch_scale: {f_scale:.4f}")
    print(f"write_scale: {w_scale:.4f}")
    print(f"hbm_bytes_per_launch: {hbm:.0f}")
    if args.algorithmic_bytes:
        print(f"algorithmic_bytes_per_launch: {args.algorithmic_bytes}")
        print(f"traffic_over_algorithmic: {hbm / args.algorithmic_bytes:.4f}")
    print(f"sources: {' '.join(SOURCES[args.sources])}")
    print(f"source_sha256: {source_sha256(SOURCES[args.sources])}")


def cmd_pmc(args):
    fetch = counter_per_dispatch(args.fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(args.write_db, "WRITE_SIZE")
    print(f"{'kernel':80s} {'dispatches':>10s} {'fetch_KiB':>12s} {'write_KiB':>12s} {'hbm_MB':>10s}")
    rows = []
    for k in set(fetch) | set(write):
        f, fn, _ = fetch.get(k, (0.0, 0, 0.0))
        w, wn, _ = write.get(k, (0.0, 0, 0.0))
        rows.append((k, max(fn, wn), f, w, (2.0 * f + w) * 1024.0 / 1e6))
    rows.sort(key=lambda r: -r[4])
    for k, n, f, w, mb in rows:
        print(f"{_short(k, 80):80s} {n:10d} {f:12.1f} {w:12.1f} {mb:10.2f}")


def all_counters(db: str, match: str):
    """{kernel: {counter: mean per dispatch}} for kernels containing `match`."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, counter_name, dispatch_id, sum(value) from counters_collection "
        "group by kernel_name, counter_name, dispatch_id").fetchall()
    con.close()
    agg: dict[str, dict[str, list[float]]] = {}
    for k, c, _, v in rows:
        if match in k:
            agg.setdefault(k, {}).setdefault(c, []).append(float(v))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in agg.items()}


def cmd_counters(args):
    merged: dict[str, dict[str, float]] = {}
    for db in args.dbs:
        for k, cs in all_counters(db, args.match).items():
            merged.setdefault(k, {}).update(cs)
    for k in sorted(merged):
        cs = merged[k]
        print(f"kernel: {k}")
        for c in sorted(cs):
            print(f"  {c}: {cs[c]:.6g}")
        waves = cs.get("SQ_WAVES")
        if waves and "SQ_INSTS_VALU" in cs:
            print(f"  valu_insts_per_wave: {cs['SQ_INSTS_VALU'] / waves:.1f}")
        if cs.get("SQ_WAVE_CYCLES") and "SQ_ACTIVE_INST_VALU" in cs:
            # both count in the same (quad-cycle) unit per wave
            print(f"  valu_issue_share_of_wave_time: {cs['SQ_ACTIVE_INST_VALU'] / cs['SQ_WAVE_CYCLES']:.3f}")
        if cs.get("SQ_ACTIVE_INST_LDS") and "SQ_LDS_BANK_CONFLICT" in cs:
            print(f"  lds_bank_conflict_per_lds_active: "
                  f"{cs['SQ_LDS_BANK_CONFLICT'] / cs['SQ_ACTIVE_INST_LDS']:.3f}")
        if cs.get("SQ_BUSY_CYCLES") and "SQ_VALU_MFMA_BUSY_CYCLES" in cs:
            print(f"  mfma_busy_per_sq_busy: "
                  f"{cs['SQ_VALU_MFMA_BUSY_CYCLES'] / cs['SQ_BUSY_CYCLES']:.3f}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--match")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", required=True, action="append",
                   help="substring of a kernel name; repeat to sum kernels launched together")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--algorithmic-bytes", type=int, default=0)
    t.add_argument("--sources", choices=sorted(SOURCES), default="pass1",
                   help="kernel sources whose hash the summary records")
    t.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer",
                   help="substring naming the copy kernel of known size (the runtime's "
                        "device-to-device copy by default; its largest dispatch is taken)")
    m = sub.add_parser("pmc")
    m.add_argument("fetch_db")
    m.add_argument("write_db")
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--match", required=True)
    args = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "pmc": cmd_pmc,
     "counters": cmd_counters}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
