"""Profiling driver for the fused step, run under rocprofv3 by profile_run.sh.

python -m paper_1902_08933_amd.profile_step --workload spinodal4096 --steps 20
python -m paper_1902_08933_amd.profile_step --workload spinodal1024 --autotune   (strip shape)
python -m paper_1902_08933_amd.profile_step --workload r4_1024   (Remark 4 scheme, single phase)
python -m paper_1902_08933_amd.profile_step --workload d3q15_256   (D3Q15 two-phase step)
python -m paper_1902_08933_amd.profile_step --workload batch256 --steps 40   (batched persistent step)
python -m paper_1902_08933_amd.profile_step --copy-mib 2048 --steps 10   (bandwidth probe:
    copy / read / write of a known byte count, the reference for the HBM roofline and for
    scaling the FETCH_SIZE / WRITE_SIZE counters)
"""
import argparse
import re
import sys

from . import lbpf, workloads

BYTES_PER_CELL = 160  # algorithmic bytes per node update of the D2Q9 step
BATCH_WARMUP = 1000   # warm-up of the batch, in stretches of BATCH_CHECK steps
BATCH_CHECK = 200     # the instances that went non-finite are frozen after each stretch


def warm_up_batch(b, steps=BATCH_WARMUP, every=BATCH_CHECK):
    """Advance the batch `steps` steps, freezing the instances that went non-finite after every
    `every` steps (the unstable ones, the largest density ratios, diverge at different times, the
    last ones after several hundred steps); returns the frozen flags."""
    flags = None
    for _ in range(max(1, steps // every)):
        b.step(every)
        flags, _ = b.status()
    return flags


def make(name, variant):
    if name.startswith("spinodal"):
        n = int(name[len("spinodal"):])
        return workloads.spinodal(n=n, variant=variant, seed=0)
    if name == "bubble512x2048":
        return workloads.rising_bubble(nx=512, ny=2048, R=64.0, rho_ratio=10.0, variant=variant)
    if name == "poiseuille256x128":
        return workloads.layered_poiseuille(nx=256, ny=128, variant=variant)
    raise SystemExit(f"unknown workload {name}")


def run_sp(torch, n, steps, warmup, remark4=False):
    """single-phase step with a mass source and the full force term: the incompressible model, or
    (remark4) the nearly incompressible model on the explicit D_i G_i scheme with a linear drag"""
    import numpy as np
    if remark4:
        cfg, f = workloads.single_phase_source(n, n, model="nearly_incompressible", S0=1e-4, F0=1e-6,
                                               full=True, scheme="remark4", drag=0.01)
    else:
        cfg, f = workloads.single_phase_source(n, n, model="incompressible", S0=1e-4, F0=1e-6, full=True)
    sim = lbpf.SinglePhase(cfg).init(*(torch.from_numpy(f[k].astype(np.float32)).cuda()
                                       for k in ("a0", "ux", "uy", "S", "Fx", "Fy")))
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_d3q15(torch, n, steps, warmup, shape=None):
    """D3Q15 spinodal at n^3: the autotuned (or given) launch shape, ms per step"""
    cfg, phi = workloads.spinodal3d(n=n, seed=0)
    sim = lbpf.Simulation3D(cfg).init(torch.from_numpy(phi.astype("float32")).cuda())
    s = sim.autotune(3) if shape is None else shape
    sim.set_shape(s)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return s, e0.elapsed_time(e1) / steps


def make_batch(torch, count=256, seed=0, tile=None):
    """the batched workload of the benchmark: seeded instances, the benchmark's warm-up (at strip
    shape `tile` when given, so that a profiled run launches one kernel only), unstable ones
    frozen; returns the batch, its active node count and its total node count"""
    import numpy as np
    insts = workloads.batch_instances(count, seed=seed)
    b = lbpf.Batch([c for c, _ in insts])
    if tile is not None:
        b.set_tile(tile)
    for k, (_, phi) in enumerate(insts):
        b.init(k, torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    flags = warm_up_batch(b)
    active = sum(c["nx"] * c["ny"] for c, f in zip(b.cfgs, flags) if not f)
    total = sum(c["nx"] * c["ny"] for c in b.cfgs)
    return b, active, total


def run_batch(torch, steps, warmup, tile=None):
    """graph-replayed persistent batched step: ms per step at the given (or autotuned) shape"""
    b, active, total = make_batch(torch, tile=tile)
    if tile is None:
        tile, _ = b.autotune(trial_steps=8)
    b.set_tile(tile)
    b.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return tile, e0.elapsed_time(e1) / steps, active, total


def run_steps(torch, cfg, phi, steps, warmup, tile):
    sim = lbpf.Simulation(cfg)
    if tile is not None:
        sim.set_tile(tile)
    sim.init(torch.from_numpy(phi.astype("float32")).cuda())
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="spinodal1024")
    ap.add_argument("--variant", default="qim")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, default=None, help="strip shape (default: library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="print the strip shape the library's autotuner picks for the workload and exit")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--probe-blocks", type=int, default=0)
    a = ap.parse_args()
    if a.copy_mib:
        nbytes = a.copy_mib * (1 << 20)
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for mode, name, moved in ((0, "copy", 2), (1, "read", 1), (2, "write", 1)):
            for blocks in ((a.probe_blocks,) if a.probe_blocks else (1024, 4096, 16384)):
                dst = y if mode != 1 else torch.empty(blocks, dtype=torch.float32, device="cuda")
                lbpf.bw_probe(mode, x, dst, nbytes, blocks)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(a.steps):
                    lbpf.bw_probe(mode, x, dst, nbytes, blocks)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / a.steps
                print(f"probe {name} {a.copy_mib} MiB, {blocks} workgroups: {ms:.4f} ms, "
                      f"{moved * nbytes / ms / 1e6:.1f} GB/s", flush=True)
        return
    if a.workload.startswith("d3q15_"):
        n = int(a.workload[len("d3q15_"):])
        if a.autotune:
            cfg, phi = workloads.spinodal3d(n=n, seed=0)
            sim = lbpf.Simulation3D(cfg).init(torch.from_numpy(phi.astype("float32")).cuda())
            print(sim.autotune(3), flush=True)
            return 0
        s, ms = run_d3q15(torch, n, a.steps, a.warmup, shape=a.tile)
        print(f"{a.workload} shape {s} {lbpf.shapes3d()[s]}: {ms:.4f} ms/step, "
              f"{n ** 3 / (ms * 1e-3) / 1e6:.0f} MLUPS, {264 * n ** 3 / (ms * 1e-3) / 1e9:.0f} GB/s",
              flush=True)
        return 0
    if a.workload == "batch256":
        if a.autotune:  # last line: the strip shape and the number of active nodes
            b, active, _ = make_batch(torch)
            print(b.autotune(trial_steps=8)[0], active, flush=True)
            return 0
        tile, ms, active, total = run_batch(torch, a.steps, a.warmup, a.tile)
        print(f"batch256 tile {tile} {lbpf.tile_shapes()[tile]}: {ms:.4f} ms/step, active {active} of "
              f"{total} nodes, {active / (ms * 1e-3) / 1e6:.0f} MLUPS, "
              f"{BYTES_PER_CELL * total / (ms * 1e-3) / 1e9:.0f} GB/s", flush=True)
        return 0
    single = re.fullmatch(r"(sp|r4_)(\d+)", a.workload)  # "spinodal<N>" is the two-phase step
    if single:
        r4 = single.group(1) == "r4_"
        n = int(single.group(2))
        ms = run_sp(torch, n, a.steps, a.warmup, remark4=r4)
        b = 244 if r4 else 92
        print(f"{a.workload}: {ms:.4f} ms/step, {n * n / (ms * 1e-3) / 1e6:.0f} MLUPS, "
              f"{b * n * n / (ms * 1e-3) / 1e9:.0f} GB/s", flush=True)
        return 0
    cfg, phi = make(a.workload, a.variant)
    cells = cfg["nx"] * cfg["ny"]
    if a.autotune:
        sim = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype("float32")).cuda())
        best, _ = sim.autotune(trial_steps=20)
        print(best, flush=True)
        return 0
    t = a.tile
    ms = run_steps(torch, cfg, phi, a.steps, a.warmup, t)
    gbs = BYTES_PER_CELL * cells / (ms * 1e-3) / 1e9
    shape = lbpf.tile_shapes()[t] if t is not None else "default"
    print(f"{a.workload} {a.variant} tile {t} {shape}: {ms:.4f} ms/step, "
          f"{cells / (ms * 1e-3) / 1e6:.0f} MLUPS, {gbs:.0f} GB/s ({gbs / 80:.1f}% of 8 TB/s)",
          flush=True)


if __name__ == "__main__":
    sys.exit(main())
