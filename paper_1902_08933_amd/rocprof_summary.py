"""Short text summaries of rocprofv3 results (SQLite .db output) for profiles/.

python -m paper_1902_08933_amd.rocprof_summary --trace T.db [--fetch F.db --write W.db
    --calib-fetch CF.db --calib-write CW.db --calib-bytes N --kernel strip_kernel --cells C]
    --command "..." --out profiles/NAME.txt

--trace: kernel-trace run: calls, total and average duration per kernel.
--fetch/--write: one --pmc FETCH_SIZE run and one --pmc WRITE_SIZE run of the same program;
each counter is scaled by what it reads for the bandwidth probe (probe_read_kernel /
probe_write_kernel of --calib-bytes bytes), giving HBM bytes per dispatch of --kernel.
"""
import argparse
import hashlib
import os
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_FILES = {
    # the state layout (strides) of the step is chosen in lbpf_api.cpp
    "step": [os.path.join(HERE, "csrc", n) for n in ("lbpf_kernels.hip", "lbpf_cell.hpp", "lbpf_model.hpp",
                                                     "lbpf_api.cpp")],
    "unet": [os.path.join(HERE, "csrc", n) for n in ("lbpf_unet_kernels.hip", "lbpf_unet_ops.hpp",
                                                     "lbpf_unet.cpp")],
    "sp": [os.path.join(HERE, "csrc", "lbpf_sp.hip")],
    "d3q15": [os.path.join(HERE, "csrc", n) for n in ("lbpf_d3q15.hip", "lbpf_cell.hpp")],
}


def kernel_source_hash(which="step"):
    h = hashlib.sha256()
    for p in KERNEL_FILES[which]:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace_span(db, key, last=0):
    """(dispatches, first start to last end in ns) of the kernel whose name contains key with the
    most dispatches (with last > 0: its last `last` dispatches): for back-to-back launches the span
    per launch is the time per launch as events around the whole sequence see it (consecutive
    dispatches overlap at their ends)"""
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end from kernels order by start").fetchall()
    by = {}
    for name, st, en in rows:
        if key in name:
            by.setdefault(name, []).append((st, en))
    if not by:
        raise SystemExit(f"no kernel matching {key!r}")
    v = max(by.values(), key=len)
    if last:
        v = v[-last:]
    return len(v), max(e for _, e in v) - min(s for s, _ in v)


def trace_stats(db, key=None, last=0):
    """per kernel name: (dispatches, total, mean, median) of the durations in ns; with key and
    last > 0, the kernels whose name contains key keep only their last `last` dispatches"""
    c = sqlite3.connect(db)
    rows = c.execute("select name, end - start from kernels order by start").fetchall()
    out = {}
    for name, d in rows:
        out.setdefault(name, []).append(d)
    if key and last:
        out = {k: (v[-last:] if key in k else v) for k, v in out.items()}
    return {k: (len(v), sum(v), statistics.mean(v), statistics.median(v)) for k, v in out.items()}


def pmc_values(db, counter):
    """per kernel name: the counter's value per dispatch, in dispatch order"""
    c = sqlite3.connect(db)
    cols = {r[1] for r in c.execute("pragma table_info(counters_collection)").fetchall()}
    order = next((k for k in ("dispatch_id", "correlation_id", "start") if k in cols), "rowid")
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ? "
                     f"order by {order}", (counter,)).fetchall()
    out = {}
    for name, v in rows:
        out.setdefault(name, []).append(v)
    return out


def pick(d, key):
    """the kernel whose name contains `key` with the most dispatches"""
    ks = [k for k in d if key in k]
    if not ks:
        raise SystemExit(f"no kernel matching {key!r} in {list(d)[:5]}")
    k = max(ks, key=lambda n: d[n][0] if isinstance(d[n], tuple) else len(d[n]))
    return k, d[k]


def bench_line(path):
    """the last JSON line a bench.py run printed, or None"""
    import json
    found = None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"ms_per_step"' in line:
                try:
                    found = json.loads(line)
                except ValueError:
                    pass
    return found


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-fetch")
    ap.add_argument("--calib-write")
    ap.add_argument("--calib-bytes", type=int, default=0)
    ap.add_argument("--kernel", default="strip_kernel")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--alg-bytes-per-cell", type=float, default=160.0)
    ap.add_argument("--storage-bytes-per-cell", type=float, default=0.0,
                    help="bytes per node the kernel stores and reloads, when above the algorithmic ones")
    ap.add_argument("--iterations", type=int, default=0,
                    help="with --trace: report the summed kernel time per iteration of the program")
    ap.add_argument("--flop", type=float, default=0.0, help="with --iterations: FLOP per iteration")
    ap.add_argument("--sources", default="step", choices=sorted(KERNEL_FILES),
                    help="which kernel sources the summary's hash covers")
    ap.add_argument("--last", type=int, default=0,
                    help="count only the last N dispatches of --kernel (the timed ones, after a "
                         "warm-up whose launches differ)")
    ap.add_argument("--bench-log", default="",
                    help="stdout of a bench.py run under the trace: its JSON line's ms_per_step is "
                         "reported beside the traced average duration of --kernel")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    lines = [f"# rocprofv3 summary", f"command: {a.command}",
             f"kernel_sources: {a.sources}", f"kernel_source_sha256_16: {kernel_source_hash(a.sources)}"]
    if a.cells:
        lines.append(f"cells: {a.cells}")
    if a.trace:
        lines.append("")
        lines.append("## kernel trace (durations in microseconds)")
        lines.append(f"{'calls':>6} {'total_us':>12} {'avg_us':>10} {'median_us':>10}  kernel")
        stats = trace_stats(a.trace, a.kernel, a.last)
        for k, (n, tot, avg, med) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
            lines.append(f"{n:6d} {tot / 1e3:12.1f} {avg / 1e3:10.3f} {med / 1e3:10.3f}  {k[:110]}")
        if a.iterations:
            # with --last, the kernels matching --kernel that ran at least once per timed
            # iteration (their last dispatches); otherwise every kernel of the program
            total = sum(v[1] for k, v in stats.items()
                        if not a.last or (a.kernel in k and v[0] >= a.iterations)) / a.iterations
            if a.last:
                lines.append(f"counted: the last {a.last} dispatches of each kernel matching {a.kernel!r} "
                             f"that runs every iteration")
            lines.append(f"total_kernel_us_per_iteration: {total / 1e3:.3f}")
            if a.flop:
                lines.append(f"flop_per_iteration: {a.flop:.6e}")
                lines.append(f"TFLOPs_at_total: {a.flop / (total * 1e-9) / 1e12:.1f}")
        if a.cells:
            name, (n, tot, avg, med) = pick(stats, a.kernel)
            gbs = a.alg_bytes_per_cell * a.cells / (avg * 1e-9) / 1e9
            n_span, span = trace_span(a.trace, a.kernel, a.last)
            if a.last:
                lines.append(f"counted: the last {a.last} dispatches of {a.kernel}")
            lines.append(f"avg_duration_us_{a.kernel}: {avg / 1e3:.3f}")
            lines.append(f"span_us_per_launch_{a.kernel}: {span / n_span / 1e3:.3f} "
                         f"(first start to last end over {n_span} back-to-back launches)")
            lines.append(f"algorithmic_bytes_per_cell: {a.alg_bytes_per_cell:.0f}")
            lines.append(f"algorithmic_GBs_at_avg_duration: {gbs:.1f}")
            lines.append(f"algorithmic_GBs_at_span: {a.alg_bytes_per_cell * a.cells / (span / n_span * 1e-9) / 1e9:.1f}")
            if a.bench_log:
                bench = bench_line(a.bench_log)
                if bench is not None:
                    bms = bench["ms_per_step"] * 1e3
                    lines.append(f"bench_ms_per_step_us: {bms:.3f} (the same run's bench.py JSON line: "
                                 f"value {bench['value']} {bench['unit']}, strip {bench['config'].get('strip')})")
                    lines.append(f"trace_avg_over_bench: {avg / 1e3 / bms:.4f}; "
                                 f"trace_span_over_bench: {span / n_span / 1e3 / bms:.4f}")
    if a.fetch and a.write:
        fk, fv = pick(pmc_values(a.fetch, "FETCH_SIZE"), a.kernel)
        wk, wv = pick(pmc_values(a.write, "WRITE_SIZE"), a.kernel)
        if a.last:
            fv, wv = fv[-a.last:], wv[-a.last:]
        f_kib, w_kib = statistics.median(fv), statistics.median(wv)
        fs = ws = 1.0
        if a.calib_fetch and a.calib_write and a.calib_bytes:
            _, cf = pick(pmc_values(a.calib_fetch, "FETCH_SIZE"), "probe_read_kernel")
            _, cw = pick(pmc_values(a.calib_write, "WRITE_SIZE"), "probe_write_kernel")
            fs = a.calib_bytes / (statistics.median(cf) * 1024)
            ws = a.calib_bytes / (statistics.median(cw) * 1024)
        hbm = f_kib * 1024 * fs + w_kib * 1024 * ws
        lines += ["", "## HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)",
                  f"kernel: {fk[:110]}",
                  f"FETCH_SIZE_KiB_median: {f_kib:.0f} (dispatches: {len(fv)})",
                  f"WRITE_SIZE_KiB_median: {w_kib:.0f} (dispatches: {len(wv)})",
                  f"calibration_probe_bytes: {a.calib_bytes}",
                  f"fetch_scale: {fs:.4f}", f"write_scale: {ws:.4f}",
                  f"hbm_bytes_per_launch: {hbm:.6e}"]
        if a.cells:
            st = f", stored {a.storage_bytes_per_cell:.0f}" if a.storage_bytes_per_cell else ""
            lines.append(f"hbm_bytes_per_cell: {hbm / a.cells:.2f} "
                         f"(read {f_kib * 1024 * fs / a.cells:.2f}, write {w_kib * 1024 * ws / a.cells:.2f}; "
                         f"algorithmic {a.alg_bytes_per_cell:.0f}{st})")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
