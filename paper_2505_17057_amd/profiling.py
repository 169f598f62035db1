"""Summaries of rocprofv3 result databases (SQLite, ``*_results.db``).

Turns one kernel-trace run and two counter runs (``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE``, each with ``--kernel-trace``) of the same program into
* a short text summary (per-kernel call count and durations, per-dispatch
  HBM counters of the step kernel and of a device copy of known size), and
* a JSON record of the step kernel's HBM bytes per launch, scaled by what the
  same counters read for the copy, keyed by the SHA-256 of the kernel source so
  that a reader can tell when the figures are stale.

The copy calibrates the counters: a device-to-device copy of B bytes moves
exactly B bytes in and B bytes out of HBM, so counter_bytes * (B / reading) is
the HBM traffic.  On gfx950 FETCH_SIZE reads half the bytes a copy fetches and
WRITE_SIZE reads them exactly; the factors are measured, not assumed.

Usage:
  python -m paper_2505_17057_amd.profiling --trace T.db --fetch F.db --write W.db \
      --kernel k_lcde_tb --copy-bytes 268435456 --kernel-source SRC --bench-log LOG \
      --algorithmic-bytes-per-step B --pass-bytes P --workload TEXT \
      --out-md profiles/X.md --out-json profiles/X.json --command "..." ...
(paper_2505_17057_amd/profile_headline.sh runs the three profiles and this.)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import shlex
import sqlite3
import sys
import statistics
from collections import defaultdict


def kernel_stats(db_path):
    """[(name, calls, total_ns, mean_ns, min_ns, max_ns)] sorted by total time."""
    db = sqlite3.connect(db_path)
    rows = defaultdict(list)
    for name, dur in db.execute("select name, duration from kernels"):
        rows[name].append(int(dur))
    out = [(n, len(d), sum(d), sum(d) / len(d), min(d), max(d)) for n, d in rows.items()]
    out.sort(key=lambda r: -r[2])
    return out


def kernel_grids(db_path, kernel):
    """{grid_x: (calls, mean_ns)} of dispatches whose name contains `kernel`."""
    db = sqlite3.connect(db_path)
    g = defaultdict(list)
    for name, grid, dur in db.execute("select name, grid_x, duration from kernels"):
        if kernel in name:
            g[int(grid)].append(int(dur))
    return {k: (len(v), sum(v) / len(v)) for k, v in g.items()}


def counter_by_grid(db_path, counter, kernel):
    """{grid: [value per dispatch]} (KiB) for dispatches whose name contains `kernel`."""
    db = sqlite3.connect(db_path)
    g = defaultdict(list)
    q = "select kernel_name, grid_size, value from counters_collection where counter_name = ?"
    for name, grid, val in db.execute(q, (counter,)):
        if kernel in name:
            g[int(grid)].append(float(val))
    return g


def copy_factor(db_path, counter, copy_bytes):
    """Scale factor bytes / (counter KiB * 1024) from the copy dispatches of
    `copy_bytes` bytes: a copy moves its bytes once each way, and the counters
    read between a quarter of them and all of them (gfx950's FETCH_SIZE reads
    half), so larger copies of the same run (state copies) are left out."""
    vals = []
    for vs in counter_by_grid(db_path, counter, "copyBuffer").values():
        vals += [v for v in vs if copy_bytes / 4 <= v * 1024.0 <= 1.25 * copy_bytes]
    if not vals:
        raise SystemExit("no copy dispatch of %d bytes found for %s" % (copy_bytes, counter))
    return copy_bytes / (statistics.fmean(vals) * 1024.0), vals


def bench_plan(log_path):
    """(tb, h, w, launch_ms_mean) from the JSON line a bench run printed."""
    for line in open(log_path):
        line = line.strip()
        if line.startswith("{") and '"roofline"' in line:
            r = json.loads(line)["roofline"]
            return (r["time_steps_per_launch"], r.get("window_rows", 0), r.get("window_cols", 64),
                    r.get("launch_ms_mean"))
    raise SystemExit("no bench JSON line in " + log_path)


def kernel_stats_by_grid(db_path):
    """[(name [grid], calls, total_ns, mean_ns, min_ns, max_ns)] per kernel and
    launch grid (a launch plan), sorted by total time."""
    db = sqlite3.connect(db_path)
    rows = defaultdict(list)
    for name, grid, dur in db.execute("select name, grid_x, duration from kernels"):
        base = name.replace("(anonymous namespace)::", "").split("(")[0]
        rows["%s [grid %d]" % (base, int(grid))].append(int(dur))
    out = [(n, len(d), sum(d), sum(d) / len(d), min(d), max(d)) for n, d in rows.items()]
    out.sort(key=lambda r: -r[2])
    return out


def stats_table(db_path, top=15, by_grid=False):
    """Markdown table of the `top` kernels by total time (per launch grid, i.e.
    per launch plan, when by_grid)."""
    stats = kernel_stats_by_grid(db_path) if by_grid else kernel_stats(db_path)
    total = sum(r[2] for r in stats) or 1
    L = ["| kernel | calls | total ms | mean us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for n, c, t, m, lo, hi in stats[:top]:
        L.append("| %s | %d | %.3f | %.3f | %.3f | %.3f | %.1f%% |" % (n[:100], c, t / 1e6, m / 1e3, lo / 1e3,
                                                                    hi / 1e3, 100.0 * t / total))
    return "\n".join(L)


def counters_table(db_paths, pattern):
    """Markdown table: per kernel (name containing `pattern`) and launch grid,
    the dispatch count and the mean per dispatch of every counter the result
    databases hold (raw values: KiB for FETCH_SIZE / WRITE_SIZE)."""
    acc = defaultdict(lambda: defaultdict(list))
    names = set()
    for path in db_paths:
        db = sqlite3.connect(path)
        q = "select kernel_name, grid_size, counter_name, value from counters_collection"
        for name, grid, cn, val in db.execute(q):
            if pattern in name:
                acc[(name, int(grid))][cn].append(float(val))
                names.add(cn)
    cols = sorted(names)
    out = ["| kernel [grid] | dispatches | " + " | ".join(cols) + " |",
           "|---|---|" + "---|" * len(cols)]
    for (name, grid), cs in sorted(acc.items()):
        n = max(len(v) for v in cs.values())
        vals = ["%.6g" % statistics.fmean(cs[c]) if cs.get(c) else "" for c in cols]
        out.append("| %s [grid %d] | %d | %s |" % (name, grid, n, " | ".join(vals)))
    return "\n".join(out)


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "counters":
        # python -m paper_2505_17057_amd.profiling counters PATTERN DB [DB ...]
        print(counters_table(argv[2:], argv[1]))
        return
    if argv and argv[0] == "stats":
        # python -m paper_2505_17057_amd.profiling stats RESULTS.db [TOP] [TITLE] [COMMAND]
        top = int(argv[2]) if len(argv) > 2 else 15
        if len(argv) > 3:
            print("# rocprofv3 kernel trace: %s\n" % argv[3])
        if len(argv) > 4:
            print("Command (from the repository root; `cd /tmp && export TMPDIR=/tmp` first):\n")
            print("    " + argv[4] + "\n")
        print(stats_table(argv[1], top, by_grid=True))
        return
    p = argparse.ArgumentParser()
    p.add_argument("--trace", required=True)
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--copy-bytes", type=int, required=True, help="bytes copied by one calibration copy")
    p.add_argument("--kernel-source", required=True)
    p.add_argument("--bench-log", default="",
                   help="log of the traced bench run (its roofline names the timed plan)")
    p.add_argument("--plan", default="",
                   help="TB,H,W of the timed plan, for runs whose log carries no roofline")
    p.add_argument("--more", action="append", default=[],
                   help="result database of a further counter run (every counter it holds for the "
                        "kernel's timed grid is listed)")
    p.add_argument("--algorithmic-bytes-per-step", type=float, required=True,
                   help="algorithmic bytes of one time step over the grid (x time steps per launch)")
    p.add_argument("--pass-bytes", type=float, required=True,
                   help="bytes of one read and one write of every stored field (the least any launch moves)")
    p.add_argument("--workload", required=True)
    p.add_argument("--out-md", required=True)
    p.add_argument("--out-json", required=True)
    p.add_argument("--command", action="append", default=[], help="command that produced an input")
    p.add_argument("--alt", action="append", default=[],
                   help="TB,H,W:FETCH_DB:WRITE_DB, counter runs of another launch plan of the kernel")
    p.add_argument("--valu", default="",
                   help="result database of a run with --pmc SQ_INSTS_VALU SQ_WAVES (optional)")
    p.add_argument("--flops-per-lup", type=float, default=0.0,
                   help="algorithmic flops per lattice update (for the VALU summary)")
    p.add_argument("--lups-per-step", type=float, default=0.0,
                   help="lattice updates of one time step over the grid")
    a = p.parse_args(argv)
    here = os.getcwd() + os.sep
    a.command = a.command + ["python -m paper_2505_17057_amd.profiling " +
                             shlex.join(x.replace(here, "") for x in argv)]

    stats = kernel_stats(a.trace)
    grids = kernel_grids(a.trace, a.kernel)
    if a.plan:
        tb, h, w = (int(v) for v in a.plan.split(","))
        ev_ms = None
    else:
        tb, h, w, ev_ms = bench_plan(a.bench_log)
    a.algorithmic_bytes = a.algorithmic_bytes_per_step * tb
    ff, fvals = copy_factor(a.fetch, "FETCH_SIZE", a.copy_bytes)
    wf, wvals = copy_factor(a.write, "WRITE_SIZE", a.copy_bytes)
    # the counter runs launch the timed plan only (no autotuning), so its grid
    # is the one they launch most; the trace's autotuning scan launches other
    # grids, some of them more often than the timed plan's
    fgrids = counter_by_grid(a.fetch, "FETCH_SIZE", a.kernel)
    main_grid = max(fgrids, key=lambda g: len(fgrids[g]))
    if main_grid not in grids:
        raise SystemExit("the trace has no launch of the counter runs' grid %d" % main_grid)
    fk = fgrids[main_grid]
    wk = counter_by_grid(a.write, "WRITE_SIZE", a.kernel)[main_grid]
    fetch_b = statistics.fmean(fk) * 1024.0 * ff
    write_b = statistics.fmean(wk) * 1024.0 * wf
    traffic = fetch_b + write_b
    sha = hashlib.sha256(open(a.kernel_source, "rb").read()).hexdigest()
    calls, mean_ns = grids[main_grid]
    rec = dict(kernel=a.kernel, workload=a.workload, kernel_source=a.kernel_source,
               kernel_source_sha256=sha, time_steps_per_launch=tb, window_rows=h, window_cols=w,
               grid_threads=main_grid, dispatches=calls, trace_mean_us=round(mean_ns / 1e3, 3),
               fetch_kib_raw=statistics.fmean(fk), write_kib_raw=statistics.fmean(wk),
               fetch_factor=round(ff, 5), write_factor=round(wf, 5),
               hbm_bytes_per_launch=round(traffic), algorithmic_bytes_per_launch=a.algorithmic_bytes,
               one_pass_bytes=a.pass_bytes,
               commands=a.command)
    # other plans the autotuner may pick: their counters, scaled the same way
    alts = []
    for spec in a.alt:
        plan, fdb, wdb = spec.split(":")
        atb, ah, aw = (int(v) for v in plan.split(","))
        fg = counter_by_grid(fdb, "FETCH_SIZE", a.kernel)
        wg = counter_by_grid(wdb, "WRITE_SIZE", a.kernel)
        g = max(fg, key=lambda k: len(fg[k]))
        afk, awk = fg[g], wg[g]
        ab = statistics.fmean(afk) * 1024.0 * ff + statistics.fmean(awk) * 1024.0 * wf
        alts.append(dict(time_steps_per_launch=atb, window_rows=ah, window_cols=aw,
                         hbm_bytes_per_launch=round(ab), fetch_kib_raw=statistics.fmean(afk),
                         write_kib_raw=statistics.fmean(awk), dispatches=len(afk)))
    rec["alternates"] = alts
    valu = None
    if a.valu:
        vg = counter_by_grid(a.valu, "SQ_INSTS_VALU", a.kernel)
        wg = counter_by_grid(a.valu, "SQ_WAVES", a.kernel)
        if main_grid in vg:
            vi = statistics.fmean(vg[main_grid])
            wv = statistics.fmean(wg[main_grid]) if main_grid in wg else None
            valu = dict(insts=vi, waves=wv, dispatches=len(vg[main_grid]))
            rec["valu_insts_per_launch"] = round(vi)
            rec["waves_per_launch"] = round(wv) if wv else None
    more = []
    for db in a.more:
        con = sqlite3.connect(db)
        q = "select distinct counter_name from counters_collection"
        for (cn,) in con.execute(q):
            g = counter_by_grid(db, cn, a.kernel)
            if main_grid in g:
                more.append((cn, statistics.fmean(g[main_grid]), len(g[main_grid])))
    if more:
        rec["counters"] = {cn: v for cn, v, _ in more}
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")

    L = []
    L.append("# rocprofv3 summary: %s, %s\n" % (a.kernel, a.workload))
    L.append("Commands (from the repository root on the GPU box; `cd /tmp && export TMPDIR=/tmp` "
             "first, output directories under gpurun_out/):\n")
    for c in a.command:
        L.append("    " + c)
    L.append("")
    L.append("## Kernel trace (`--kernel-trace --stats`)\n")
    L.append("| kernel | calls | mean us | min us | max us | share |")
    L.append("|---|---|---|---|---|---|")
    total = sum(r[2] for r in stats) or 1
    for n, c, t, m, lo, hi in stats[:10]:
        L.append("| %s | %d | %.3f | %.3f | %.3f | %.1f%% |" % (n[:90], c, m / 1e3, lo / 1e3, hi / 1e3,
                                                               100.0 * t / total))
    L.append("")
    L.append("Timed plan of `%s`: %d time steps per launch, LDS window %d x %d (rows x columns), "
             "grid %d threads, %d dispatches, mean %.3f us (trace); the bench's own HIP-event mean "
             "over its timed region: %s us.\n" % (a.kernel, tb, h, w, main_grid, calls, mean_ns / 1e3,
                                  "%.3f" % (ev_ms * 1e3) if ev_ms else "n/a"))
    L.append("## HBM counters (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`, KiB per dispatch)\n")
    L.append("| dispatch | FETCH_SIZE KiB | WRITE_SIZE KiB |")
    L.append("|---|---|---|")
    L.append("| copy of %d B (mean of %d/%d) | %.1f | %.1f |" % (a.copy_bytes, len(fvals), len(wvals),
                                                             statistics.fmean(fvals), statistics.fmean(wvals)))
    L.append("| %s, timed plan (mean of %d/%d) | %.1f | %.1f |" % (a.kernel, len(fk), len(wk),
                                                                 statistics.fmean(fk), statistics.fmean(wk)))
    L.append("")
    L.append("Copy calibration: FETCH factor %.4f, WRITE factor %.4f (bytes moved / counter bytes)." % (ff, wf))
    L.append("Scaled HBM traffic per launch: read %.0f B + write %.0f B = %.0f B, i.e. %.3f x one pass "
             "over the stored fields (%.0f B) and %.3f x the algorithmic bytes of the launch's time steps "
             "(%.0f B)." % (fetch_b, write_b, traffic, traffic / a.pass_bytes, a.pass_bytes,
                            traffic / a.algorithmic_bytes, a.algorithmic_bytes))
    if alts:
        L.append("")
        L.append("Other launch plans of the same kernel (the same counters and factors):\n")
        L.append("| plan (TB, rows, cols) | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch | x one pass |")
        L.append("|---|---|---|---|---|")
        for r in alts:
            L.append("| %d, %d, %d | %.1f | %.1f | %d | %.3f |" % (
                r["time_steps_per_launch"], r["window_rows"], r["window_cols"], r["fetch_kib_raw"],
                r["write_kib_raw"], r["hbm_bytes_per_launch"], r["hbm_bytes_per_launch"] / a.pass_bytes))
        L.append("")
    if valu:
        dur_s = mean_ns * 1e-9
        issue = valu["insts"] / (dur_s * 256 * 2.4e9)
        L.append("## VALU issue (`--pmc SQ_INSTS_VALU SQ_WAVES`)\n")
        L.append("| quantity | per launch |")
        L.append("|---|---|")
        L.append("| SQ_INSTS_VALU (wavefront instructions, mean of %d) | %.0f |" % (valu["dispatches"],
                                                                                 valu["insts"]))
        if valu["waves"]:
            L.append("| SQ_WAVES | %.0f |" % valu["waves"])
            L.append("| VALU instructions per wavefront | %.1f |" % (valu["insts"] / valu["waves"]))
        if a.lups_per_step:
            L.append("| VALU instructions per lattice update (x 64 lanes) | %.1f |"
                     % (valu["insts"] * 64 / (a.lups_per_step * tb)))
        L.append("")
        L.append("VALU issue rate over the trace's mean launch: %.3e wavefront instructions/s, "
                 "%.3f wavefront instructions per CU per clock (256 CUs, 2.4 GHz)." %
                 (valu["insts"] / dur_s, issue))
        if a.flops_per_lup and a.lups_per_step:
            tf = a.flops_per_lup * a.lups_per_step * tb / dur_s / 1e12
            L.append("Algorithmic flops (%.0f per update): %.2f TFLOP/s = %.3f of the published FP32 "
                     "vector peak (157.3 TFLOP/s)." % (a.flops_per_lup, tf, tf / 157.3))
        L.append("")
    if more:
        L.append("## Further counters (per dispatch of the timed plan)\n")
        L.append("| counter | mean per dispatch | dispatches |")
        L.append("|---|---|---|")
        for cn, v, n in more:
            L.append("| %s | %.1f | %d |" % (cn, v, n))
        L.append("")
    L.append("Kernel source SHA-256: `%s` (%s)." % (sha, a.kernel_source))
    with open(a.out_md, "w") as f:
        f.write("\n".join(L) + "\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
