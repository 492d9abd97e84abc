"""The profile summary tool on a synthetic kernel-trace database (no GPU): per-kernel statistics,
the per-iteration kernel time of a program with warm-up passes, and the last-N selection."""
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _trace_db(path, runs):
    """runs: [(kernel name, [durations in ns])], dispatched back to back in list order per kernel,
    kernels interleaved by iteration"""
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, start integer, end integer)")
    t = 0
    longest = max(len(d) for _, d in runs)
    for i in range(longest):
        for name, durs in runs:
            if i < len(durs):
                c.execute("insert into kernels values (?, ?, ?)", (name, t, t + durs[i]))
                t += durs[i] + 10
    c.commit()
    c.close()


def _summary(tmp_path, db, *args):
    out = tmp_path / "summary.txt"
    subprocess.run([sys.executable, "-m", "paper_1902_08933_amd.rocprof_summary", "--trace", str(db),
                    "--sources", "unet", "--out", str(out), *args], check=True, cwd=ROOT)
    return out.read_text()


def _value(text, key):
    line = next(l for l in text.splitlines() if l.startswith(key + ":"))
    return float(line.split(":", 1)[1].split()[0])


@pytest.fixture
def warm_trace(tmp_path):
    # two per-pass kernels: 5 warm-up passes at 2x the time, then 10 timed passes; one setup
    # kernel that runs once
    db = tmp_path / "trace.db"
    _trace_db(db, [("void lbpf::conv_a(int)", [2000] * 5 + [1000] * 10),
                   ("void lbpf::conv_b(int)", [4000] * 5 + [3000] * 10),
                   ("void lbpf::setup_kernel(int)", [500]),
                   ("at::native::fill_kernel", [700])])
    return db


def test_per_iteration_time_counts_only_the_timed_passes_of_the_library_kernels(tmp_path, warm_trace):
    text = _summary(tmp_path, warm_trace, "--iterations", "10", "--kernel", "lbpf::", "--last", "10",
                    "--flop", "4e12")
    # last 10 dispatches of conv_a (1 us) and conv_b (3 us); the once-run kernels are not counted
    assert _value(text, "total_kernel_us_per_iteration") == pytest.approx(4.0)
    assert _value(text, "TFLOPs_at_total") == pytest.approx(4e12 / 4e-6 / 1e12, rel=1e-3)
    # the per-kernel table shows the kept dispatches
    row = next(l for l in text.splitlines() if "lbpf::conv_b" in l)
    assert row.split()[0] == "10" and float(row.split()[2]) == pytest.approx(3.0)


def test_without_last_every_dispatch_of_every_kernel_counts(tmp_path, warm_trace):
    text = _summary(tmp_path, warm_trace, "--iterations", "15")
    total_ns = 5 * 2000 + 10 * 1000 + 5 * 4000 + 10 * 3000 + 500 + 700
    assert _value(text, "total_kernel_us_per_iteration") == pytest.approx(total_ns / 15 / 1e3, abs=1e-3)
