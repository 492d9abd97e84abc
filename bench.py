"""Benchmark of the fused phase-field LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload spinodal1024|spinodal4096]

A step is one time step of the coupled D2Q9 solver (pull of the stored populations, phi/mu
stencils, forces, eq. (28) pressure, both collisions, push-streaming) over the whole grid: one
launch of the fused kernel. Inputs are synthetic (seeded spinodal noise), resident in HBM when
the timed region starts. Prints one JSON line.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic HBM bytes per node update of the method: the hydrodynamic populations 1..8 (the rest
# population is never read), the nine phase-field populations, p^{n-1} and (phi u)^{n-1}, each
# FP32 read once and written once: 20 + 20 values.
BYTES_PER_CELL = 160
# What the kernel stores per node and step on top: the low word of the rest phase-field
# population (an FP32 hi/lo pair), read and written: 21 + 21 values.
STORAGE_BYTES_PER_CELL = 168
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
FWD_WARMUP = 100       # untimed U-Net forward passes before the timed ones (the clocks settle)
ROOFLINE_GATE = 0.70   # target fraction of the peak, judged at a footprint far above the 256 MB cache


def traffic_summary_path(workload, prefix="fused_step"):
    return os.path.join(ROOT, "profiles", f"{prefix}_{workload}_pmc.txt")


def measured_traffic(workload, cells, tile, prefix="fused_step", sources="step"):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it was taken on the
    current kernel source with the same strip (launch) shape (tile None: a kernel without
    shapes); otherwise None."""
    from paper_1902_08933_amd.rocprof_summary import kernel_source_hash
    path = traffic_summary_path(workload, prefix)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    c = re.search(r"cells:\s*([0-9]+)", text)
    k = re.search(r"--tile (\d+)", text)
    if not (m and t and c) or m.group(1) != kernel_source_hash(sources) or int(c.group(1)) != cells:
        return None
    if tile is not None and (not k or int(k.group(1)) != tile):
        return None
    return float(t.group(1))


def workload(name, variant):
    from paper_1902_08933_amd import workloads as W
    if name == "spinodal1024":
        return W.spinodal(n=1024, variant=variant, seed=0)
    if name == "spinodal4096":
        return W.spinodal(n=4096, variant=variant, seed=0)
    raise SystemExit(f"unknown workload {name}")


def time_gpu(cfg, phi, steps, warmup, tile=None):
    """Time `steps` steps after `warmup`; the strip shape is `tile`, else the one the library's
    autotuner picks on this grid (it restores the state it ran on)."""
    import torch
    from paper_1902_08933_amd import lbpf
    sim = lbpf.Simulation(cfg)
    sim.init(torch.from_numpy(phi.astype("float32")).cuda())
    if tile is not None:
        sim.set_tile(tile)
    else:
        sim.autotune(trial_steps=20)
    sim.step(warmup)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    diag = sim.diagnostics()
    return ms, wall, diag, lbpf.tile_shapes()[sim.tile], sim.tile


def probe_copy_gbs(mib=2048, reps=10):
    """Bandwidth probe (plain 16-byte copy kernel): the practical HBM reference on this GPU."""
    import torch
    from paper_1902_08933_amd import lbpf
    nbytes = mib << 20
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    best = 0.0
    for blocks in (512, 1024, 2048):
        lbpf.bw_probe(0, x, y, nbytes, blocks)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lbpf.bw_probe(0, x, y, nbytes, blocks)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del x, y
    return best




def batch_bench(steps, count=256, seed=0):
    """256 independent instances (sides 64..512): one graph-replayed persistent launch per step
    vs one single-simulation launch per instance per step. Instances the method cannot hold
    stable (the largest density ratios) are frozen after a warm-up past their divergence window;
    MLUPS counts the nodes of the instances that are still finite at the end of the run (the
    frozen count is taken again after the timed legs, and the legs are re-timed if it grew)."""
    import numpy as np
    import torch
    from paper_1902_08933_amd import lbpf
    from paper_1902_08933_amd import workloads as W
    from paper_1902_08933_amd.profile_step import BATCH_WARMUP, warm_up_batch
    insts = W.batch_instances(count, seed=seed)
    b = lbpf.Batch([c for c, _ in insts])
    for k, (_, phi) in enumerate(insts):
        b.init(k, torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    del insts
    flags = warm_up_batch(b)  # freezes the instances that went unstable
    frozen_warm = int(sum(flags))
    b.autotune(trial_steps=8)  # strip shape for the active instances
    total = sum(c["nx"] * c["ny"] for c in b.cfgs)
    ratio = [c["rho_A"] / c["rho_B"] for c in b.cfgs]
    out = {"instances": count, "warmup_steps": BATCH_WARMUP, "frozen_after_warmup": frozen_warm,
           "total_nodes": total, "strip": list(lbpf.tile_shapes()[b.tile]),
           "density_ratio_ge_150": {"instances": int(sum(r >= 150 for r in ratio)),
                                    "node_fraction": round(sum(c["nx"] * c["ny"] for c, r in zip(b.cfgs, ratio)
                                                               if r >= 150) / total, 3)}}

    def timed(fn):
        fn(8)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the per-instance reference runs at its own best strip shape (a shape good for one persistent
    # launch over every instance is not the best for a launch per small instance)
    batch_tile = b.tile
    for attempt in range(2):
        per_inst = {}
        for t in sorted({batch_tile, 0, 1, 5, 12}):
            b.set_tile(t)
            per_inst[t] = timed(b.step_each)
        best_each = min(per_inst, key=per_inst.get)
        b.set_tile(batch_tile)
        ms_graph = timed(b.step)
        flags_end, _ = b.status()
        if int(sum(flags_end)) == int(sum(flags)):
            break
        flags = flags_end  # an instance went non-finite during the timed legs: time again
    active = sum(c["nx"] * c["ny"] for c, f in zip(b.cfgs, flags_end) if not f)
    out.update({"frozen": int(sum(flags_end)), "frozen_at_end": int(sum(flags_end)), "active_nodes": active,
                "steps_total": int(b.step_count)})
    out["launch_per_instance_strip"] = list(lbpf.tile_shapes()[best_each])
    for name, ms in (("graph_persistent", ms_graph), ("launch_per_instance", per_inst[best_each])):
        # frozen instances leave the work list, so only the active nodes move bytes
        gbs = BYTES_PER_CELL * active / (ms * 1e-3) / 1e9
        out[name] = {"ms_per_step": round(ms, 4), "MLUPS": round(active / (ms * 1e-3) / 1e6, 1),
                     "algorithmic_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["speedup"] = round(out["launch_per_instance"]["ms_per_step"] / out["graph_persistent"]["ms_per_step"], 2)
    # HBM bytes of one persistent launch, from the committed counter summary of this workload
    out["graph_persistent"]["traffic"] = measured_traffic("batch256", active, batch_tile, prefix="batch_step")
    return out


def unet_flops(net, h, w):
    """multiply-add FLOPs of one forward pass (2 per MAC) at h x w from the layer table"""
    f = 0
    for i, l in enumerate(net.layers()):
        level = {0: 0, 1: 1, 2: 2, 3: 3, 4: 2, 5: 1, 6: 0, 7: 0}[i]
        pix = (h >> level) * (w >> level)
        f += 2 * pix * l["cout"] * l["ks"] ** 2 * l["cin"]
    return f


SURROGATE_SEEDS = (1001, 1002, 1003)  # held out: the training trajectories use seeds 0..255


def surrogate_bench(train_steps=20000, cycles=20, seeds=SURROGATE_SEEDS, n_traj=256):
    """The learned surrogate at the scale of its workload: trained on 2 x n_traj seeded 256^2
    trajectories of the solver (spinodal runs recorded from t = 1000 to 11000 and droplet
    mergers from t = 200 to 5200, every 50 steps), then the hybrid (9 network strides of 50 steps
    + one 50-step LB stride per 500 steps, with fallback) against the plain LB on the 1024^2
    spinodal from t = 1000 over `cycles` cycles (10^4 steps) on held-out seeds; per cycle the phi
    and u errors of the hybrid, of the LB with the hybrid's hand-over but no network (control),
    and of the 2x coarser LB, and the speedups."""
    import numpy as np
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    t0 = time.perf_counter()
    store = S.generate_store(n=256, n_spinodal=n_traj, n_merger=n_traj, spinodal_t=(1000, 11000),
                             merger_t=(200, 5200))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    hold = rng.random(store.npairs) < 0.02
    net = lbpf.UNet(max_batch=8, max_h=256, max_w=256, train=True, seed=1)
    t0 = time.perf_counter()
    losses = S.train_store(net, store, steps=train_steps, batch=8, lr=5e-4, loss_weights=[4.0, 1.0, 1.0, 1.0],
                           holdout=hold)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # one-stride error on held-out pairs of the spinodal trajectories, per channel, against
    # persistence (x(t + 50) ~ x(t), the method without the network)
    hi = np.nonzero(hold & (store.pairs[:, 0] == 0))[0][:128]
    e_net, e_pers = np.zeros(4), np.zeros(4)
    for i in range(0, len(hi), 8):
        x, y = store.batch(hi[i:i + 8])
        e_net += ((net.forward(x) - y) ** 2).mean(dim=(0, 1, 2)).double().cpu().numpy() * len(hi[i:i + 8])
        e_pers += ((x - y) ** 2).mean(dim=(0, 1, 2)).double().cpu().numpy() * len(hi[i:i + 8])
    e_net /= len(hi)
    e_pers /= len(hi)
    npairs, nbytes = store.npairs, store.nbytes
    del store, x, y
    torch.cuda.empty_cache()
    big = lbpf.UNet(max_batch=1, max_h=1024, max_w=1024, train=False, seed=1)
    big.set_params(net.get_params())
    del net
    # sustained rate: normalized fields of unit scale (seeded), 100 untimed passes while the
    # clocks settle, then the median of 5 timed groups of 20
    xin = torch.randn(1, 1024, 1024, 4, generator=torch.Generator().manual_seed(7)).cuda()
    yout = torch.empty_like(xin)
    for _ in range(FWD_WARMUP):
        big.forward(xin, out=yout)
    torch.cuda.synchronize()
    groups = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            big.forward(xin, out=yout)
        e1.record()
        torch.cuda.synchronize()
        groups.append(e0.elapsed_time(e1) / 20)
    fwd_ms = float(np.median(groups))
    flops = unet_flops(big, 1024, 1024)
    del xin, yout
    per_seed = {}
    for seed in seeds:
        cfg, phi = W.spinodal(n=1024, seed=seed)
        per_seed[seed] = S.horizon_eval(big, cfg, phi, cycles=cycles, t0=1000)
    rows = []
    for c in range(cycles):
        rs = [per_seed[sd][c] for sd in seeds]
        sp = [S.speedups([r])[0] for r in rs]

        def mean(key, sub=None):
            # over the seeds whose hybrid state is still finite (see hybrid_lost)
            v = [r[key] if sub is None else r[key][sub] for r in rs]
            v = [x for x in v if np.isfinite(x)]
            return float(f"{np.mean(v):.4g}") if v else None
        rows.append({"cycle": c, "t_end": rs[0]["t_end"], "network_kept": sum(r["network_kept"] for r in rs),
                     "hybrid_lost": sum(not np.isfinite(r["hybrid"]["phi_rel_l2"]) for r in rs),
                     "lb_ms": mean("lb_ms"), "hybrid_ms": mean("hybrid_ms"), "coarse_ms": mean("coarse_ms"),
                     "hybrid_phi_rel_l2": mean("hybrid", "phi_rel_l2"), "hybrid_u_rel_l2": mean("hybrid", "u_rel_l2"),
                     "hybrid_domain_length_ratio": mean("hybrid", "domain_length_ratio"),
                     "coarse_phi_rel_l2": mean("coarse", "phi_rel_l2"), "coarse_u_rel_l2": mean("coarse", "u_rel_l2"),
                     "coarse_domain_length_ratio": mean("coarse", "domain_length_ratio"),
                     "control_phi_rel_l2": mean("control", "phi_rel_l2"), "control_u_rel_l2": mean("control", "u_rel_l2"),
                     "speedup_raw": float(f"{np.mean([x['raw'] for x in sp]):.3g}"),
                     "speedup_at_equal_phi_error": float(f"{np.mean([x['at_equal_phi_error'] for x in sp]):.3g}"),
                     "cheapest_plain_lb_at_hybrid_error": [x["alternative"] for x in sp]})
    # the horizon over which the hybrid is both faster and more accurate than the coarse LB
    held = 0
    for r in rows:
        if (r["hybrid_lost"] == 0 and r["hybrid_phi_rel_l2"] < r["coarse_phi_rel_l2"]
                and r["speedup_at_equal_phi_error"] > 1.0):
            held += 1
        else:
            break
    tot_lb = sum(r["lb_ms"] for r in rows)
    tot_hy = sum(r["hybrid_ms"] for r in rows)
    # the same horizon run through without per-cycle scoring: end-to-end time of each method
    cont = {}
    for seed in seeds:
        cfg, phi = W.spinodal(n=1024, seed=seed)
        cont[seed] = S.continuous_run(big, cfg, phi, cycles=cycles, t0=1000)
    return {"net": "U-Net 32-256 ch, %d params, BF16 weights/activations, FP32 accumulate" % big.nparam,
            "train": {"trajectories": 2 * n_traj, "pairs": npairs, "store_GB": round(nbytes / 1e9, 1),
                      "steps": train_steps, "batch": 8, "seconds_data": round(t_data, 1),
                      "seconds_train": round(t_train, 1), "final_loss": float(f"{np.mean(losses[-200:]):.4g}")},
            "one_stride_mse_normalized": {"channels": ["phi", "u_x", "u_y", "p"],
                                          "network": [float(f"{v:.3g}") for v in e_net],
                                          "persistence": [float(f"{v:.3g}") for v in e_pers]},
            "forward_1024": {"ms": round(fwd_ms, 3), "warmup_passes": FWD_WARMUP,
                             "input": "seeded N(0,1) fields, 1 x 1024 x 1024 x 4",
                             "ms_timed_groups": [round(g, 4) for g in groups], "flop": flops,
                             "TFLOPs": round(flops / (fwd_ms * 1e-3) / 1e12, 1),
                             "frac_of_bf16_peak": round(flops / (fwd_ms * 1e-3) / 2.5e15, 4)},
            "horizon": {"grid": "1024x1024 spinodal", "t_start": 1000, "cycles": cycles, "steps_per_cycle": 500,
                        "held_out_seeds": list(seeds),
                        "error_norms": "phi: ||a - b|| / ||b - mean(b)||; u: ||a - b|| / ||b||; vs the plain LB",
                        "per_cycle_mean_over_seeds": rows},
            "cycles_hybrid_faster_and_more_accurate_than_coarse_lb": held,
            "speedup_raw_over_horizon": round(tot_lb / tot_hy, 2),
            "continuous_run": {"note": "each method run through the horizon without stopping "
                                       "between cycles, timed as a whole (same hybrid decisions)",
                               "per_seed": {str(k): v for k, v in cont.items()},
                               "speedup_mean": round(float(np.mean([v["speedup"] for v in cont.values()])), 2)},
            "speedup_at_equal_phi_error_first_cycle": rows[0]["speedup_at_equal_phi_error"],
            "phi_rel_l2_first_cycle": rows[0]["hybrid_phi_rel_l2"],
            "u_rel_l2_first_cycle": rows[0]["hybrid_u_rel_l2"]}


# algorithmic bytes per node update of the single-phase step (FP32 values read + written):
# incompressible with the full force term: g_0..8, S, F_x, F_y, p^{n-1} read; g, p^n written;
# nearly incompressible: g, S, F, u^{n-1} read; g, u^n written
# Remark 4 (two passes): G pass reads f~, S, F, u^{n-1} and writes G, u; the collision reads f~,
# G(x), G(t-1) (G at the neighbours comes from L2) and writes f~
SP_BYTES = {("incompressible", True): 4 * (13 + 10), ("incompressible", False): 4 * (12 + 9),
            ("nearly_incompressible", True): 4 * (14 + 11), ("nearly_incompressible", False): 4 * (14 + 11),
            ("remark4", True): 4 * ((14 + 11) + (27 + 9))}


def single_phase_bench(n=1024, steps=2000, warmup=100):
    """The generalized single-phase model with a mass source (Sec. 2) on an n x n periodic grid
    driven by S = 1e-4 sin(2 pi x/n) cos(2 pi y/n) and a uniform force: MLUPS and the fraction of
    the HBM roofline at the step's algorithmic bytes."""
    import numpy as np
    import torch
    from paper_1902_08933_amd import lbpf, workloads as W
    out = {}
    for name, model, full, scheme in (("incompressible", "incompressible", True, "eq24"),
                                      ("nearly_incompressible", "nearly_incompressible", True, "eq24"),
                                      ("remark4", "nearly_incompressible", True, "remark4")):
        cfg, f = W.single_phase_source(n, n, model=model, S0=1e-4, F0=1e-6, full=full, scheme=scheme,
                                       drag=0.01 if scheme == "remark4" else 0.0)
        sim = lbpf.SinglePhase(cfg).init(*(torch.from_numpy(f[k].astype(np.float32)).cuda()
                                           for k in ("a0", "ux", "uy", "S", "Fx", "Fy")))
        sim.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        b = SP_BYTES[(name if scheme == "remark4" else model, full)]
        gbs = b * n * n / (ms * 1e-3) / 1e9
        sums = sim.sums()
        out[name] = {"full_force_term": full, "scheme": scheme, "drag": cfg["drag"], "ms_per_step": round(ms, 5),
                      "MLUPS": round(n * n / (ms * 1e-3) / 1e6, 1), "bytes_per_node": b,
                      "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "finite": bool(np.isfinite(sums["rho_tilde"]))}
        if name == "incompressible" and n == 1024:  # HBM bytes per launch of sp_step_kernel
            out[name]["traffic"] = measured_traffic("sp1024", n * n, None, prefix="sp_step", sources="sp")
    out["workload"] = f"single-phase source flow {n}x{n} periodic, S0 1e-4, F 1e-6, nu 1/6"
    return out


# algorithmic bytes per node of the D3Q15 step: g_1..14 (g_0 is never read), h_0..14, p and (phi u),
# read and written; the kernel also stores the low word of h_0 (272 B)
D3Q15_BYTES = 4 * 2 * (14 + 15 + 1 + 3)
D3Q15_STORAGE_BYTES = 4 * 2 * (14 + 16 + 1 + 3)


def d3q15_bench(n=256, steps=200, warmup=20):
    """The D3Q15 two-phase step on an n^3 periodic spinodal (QIM, rho ratio 3, M_phi 0.01):
    MLUPS and the fraction of the HBM roofline at 264 algorithmic bytes per node, launch shape
    from the library's autotuner."""
    import numpy as np
    import torch
    from paper_1902_08933_amd import lbpf, workloads as W
    cfg, phi = W.spinodal3d(n=n, seed=0)
    sim = lbpf.Simulation3D(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    shape = sim.autotune(3)
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cells = n ** 3
    gbs = D3Q15_BYTES * cells / (ms * 1e-3) / 1e9
    d = sim.diagnostics()
    tx, ty, cz = lbpf.shapes3d()[shape]
    return {"workload": f"spinodal {n}^3 periodic, D3Q15, QIM, rho ratio 3, nu ratio 0.1, sigma 0.03, "
                        "W 4, M_phi 0.01, tau_h 1",
            "steps": steps, "ms_per_step": round(ms, 5), "MLUPS": round(cells / (ms * 1e-3) / 1e6, 1),
            "bytes_per_node": D3Q15_BYTES, "storage_bytes_per_node": D3Q15_STORAGE_BYTES,
            "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "launch_shape": {"tx": tx, "ty": ty, "cz": cz, "index": shape, "chosen_by": "autotuner"},
            "traffic": measured_traffic(f"d3q15_{n}", cells, shape, prefix="fused_step3d", sources="d3q15"),
            "sum_phi_final": d["sum_phi"]}


def _timed_steps(sim, steps):
    """ms per step of `steps` steps between HIP events on torch's current stream"""
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def paper_workloads_bench():
    """The paper's other D2Q9 workloads at their full sizes, each with the library's default strip
    shape: the static droplet (64^2, Sec. 4.2; Laplace's law after 6000 steps), the layered channel
    (256 x 128, walls, Sec. 4.3) and the rising bubble (512 x 2048, walls, Sec. 4.4) at density
    ratio 10, where the method stays finite (at the workload's ratio 1000 it does not). Small
    grids are launch-bound, so their MLUPS are not roofline figures."""
    import numpy as np
    import torch
    from paper_1902_08933_amd import lbpf, workloads as W

    def make(cfg, phi):
        return lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())

    out = {}
    for variant in ("qim", "im"):
        cfg, phi = W.static_droplet(n=64, R=16.0, variant=variant)
        sim = make(cfg, phi)
        ms = _timed_steps(sim, 6000)
        dp = sim.laplace_dp(32.0, 32.0, 16.0)
        out[f"static_droplet_64_{variant}"] = {
            "steps": 6000, "ms_per_step": round(ms, 5), "MLUPS": round(64 * 64 / (ms * 1e-3) / 1e6, 1),
            "laplace_dP_over_sigma_by_R_minus_1": round(dp / (cfg["sigma"] / 16.0) - 1.0, 5)}
    cfg, phi = W.layered_poiseuille()
    sim = make(cfg, phi)
    ms = _timed_steps(sim, 20000)
    out["layered_poiseuille_256x128"] = {"steps": 20000, "ms_per_step": round(ms, 5),
                                         "MLUPS": round(256 * 128 / (ms * 1e-3) / 1e6, 1)}
    cfg, phi = W.rising_bubble(nx=512, ny=2048, R=64.0, rho_ratio=10.0)
    sim = make(cfg, phi)
    sim.step(100)
    ms = _timed_steps(sim, 4000)
    d = sim.diagnostics(check=False)
    out["rising_bubble_512x2048_ratio10"] = {
        "steps": 4000, "ms_per_step": round(ms, 5), "MLUPS": round(512 * 2048 / (ms * 1e-3) / 1e6, 1),
        "finite": d["nonfinite"] == 0,
        "achieved_GBs": round(BYTES_PER_CELL * 512 * 2048 / (ms * 1e-3) / 1e9, 1)}
    return out


def _oracle_steps(args):
    """one CPU worker: the FP64 oracle on the workload's own grid and field, `steps` steps;
    returns the seconds the steps took (set-up excluded)"""
    cfg, phi, steps = args
    import numpy as np
    import oracle
    o = oracle.Oracle(cfg).init(np.asarray(phi, dtype=np.float32).astype(np.float64))
    t0 = time.perf_counter()
    o.step(steps)
    return time.perf_counter() - t0


def host_cpu():
    """CPU model, logical CPUs of the host, and the CPUs this process may run on"""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, os.cpu_count(), usable


CPU_WORKERS_MAX = 16  # the host share of one GPU


def cpu_baseline(cfg, phi, steps, workers):
    """The FP64 oracle as it stands (one thread per simulation) on the workload: one simulation
    alone, then `workers` independent copies at once in separate processes (one per core). The
    all-core rate is workers x cells x steps over the slowest worker's time."""
    import multiprocessing as mp
    cells = cfg["nx"] * cfg["ny"]
    one = _oracle_steps((cfg, phi, steps))
    ctx = mp.get_context("spawn")  # fresh interpreters: the parent holds a GPU context
    with ctx.Pool(workers) as pool:
        times = pool.map(_oracle_steps, [(cfg, phi, steps)] * workers)
    return cells * steps / one / 1e6, one, workers * cells * steps / max(times) / 1e6, max(times)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="spinodal1024")
    ap.add_argument("--variant", default="qim")
    ap.add_argument("--tile", type=int, default=None, help="strip shape index (default: library default)")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-im", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-single-phase", action="store_true")
    ap.add_argument("--no-d3q15", action="store_true")
    ap.add_argument("--no-paper-workloads", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=80)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    cfg, phi = workload(args.workload, args.variant)
    cells = cfg["nx"] * cfg["ny"]
    print(f"# workload {args.workload} {cfg['nx']}x{cfg['ny']} {args.variant}: "
          f"{args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    ms, wall, diag, shape, tile = time_gpu(cfg, phi, args.steps, args.warmup, args.tile)
    ms_per_step = ms / args.steps
    mlups = cells * args.steps / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_CELL * cells / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, cells, tile)
    vname = {"qim": "QIM", "im": "IM"}[args.variant]
    out = {
        "metric": "D2Q9 two-phase MLUPS, % of HBM roofline; surrogate speedup at fixed error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded spinodal noise phi = 0.5 + U[-0.005, 0.005]",
        "config": {"workload": f"spinodal decomposition {cfg['nx']}x{cfg['ny']} periodic, "
                               f"{vname}, rho ratio 3, nu_A 0.1, nu_B 1, sigma 0.03, "
                               "W 4, M_phi 0.1, tau_h 1",
                   "nx": cfg["nx"], "ny": cfg["ny"], "variant": args.variant,
                   "strip": {"tx": shape[0], "rows": shape[1], "threads": shape[2], "index": tile,
                             "chosen_by": "set" if args.tile is not None else "autotuner"},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_cell_update": BYTES_PER_CELL,
                     "storage_bytes_per_cell_update": STORAGE_BYTES_PER_CELL,
                     "storage_frac": round(STORAGE_BYTES_PER_CELL * cells / (ms_per_step * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4),
                     "kernel": f"strip_kernel<{shape[0]},{shape[2]},{shape[1]}>",
                     "footprint_note": "the 1024^2 state (185 MB) fits the 256 MB Infinity Cache; "
                                       "large_footprint is the HBM-bound figure",
                     "copy_probe_GBs": None},
        "wall_s_timed": round(wall, 4),
        "sum_phi_final": diag["sum_phi"],
    }
    if not args.no_large and args.workload == "spinodal1024":
        # footprint far above the 256 MB Infinity Cache: 4096^2 cells, ~2.8 GB of state
        lcfg, lphi = workload("spinodal4096", args.variant)
        lsteps = max(50, args.steps // 16)
        lms, _, _, lshape, ltile = time_gpu(lcfg, lphi, lsteps, 20, args.tile)
        lcells = lcfg["nx"] * lcfg["ny"]
        lper = lms / lsteps
        lfrac = BYTES_PER_CELL * lcells / (lper * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["large_footprint"] = {
            "workload": f"spinodal 4096x4096 {vname} (2.95 GB of state)", "steps": lsteps, "ms_per_step": lper,
            "strip": {"tx": lshape[0], "rows": lshape[1], "threads": lshape[2], "index": ltile},
            "MLUPS": round(lcells / (lper * 1e-3) / 1e6, 1),
            "achieved_GBs": round(BYTES_PER_CELL * lcells / (lper * 1e-3) / 1e9, 1),
            "frac": round(lfrac, 4), "bytes_per_cell_update": BYTES_PER_CELL,
            "gate": {"frac_target": ROOFLINE_GATE, "met": bool(lfrac >= ROOFLINE_GATE)},
            "traffic": measured_traffic("spinodal4096", lcells, ltile)}
    if not args.no_im and args.workload == "spinodal1024":
        # the incompressible variant on the same grid and strip shape
        icfg, iphi = workload(args.workload, "im")
        ims, _, _, _, _ = time_gpu(icfg, iphi, args.steps, args.warmup, tile)
        iper = ims / args.steps
        out["im_variant"] = {"workload": "spinodal 1024x1024 IM", "steps": args.steps, "ms_per_step": iper,
                             "MLUPS": round(cells / (iper * 1e-3) / 1e6, 1),
                             "achieved_GBs": round(BYTES_PER_CELL * cells / (iper * 1e-3) / 1e9, 1),
                             "frac": round(BYTES_PER_CELL * cells / (iper * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["roofline"]["copy_probe_GBs"] = round(probe_copy_gbs(), 1)
    if not args.no_batch:
        out["batched"] = batch_bench(args.batch_steps)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_bench()
    if not args.no_single_phase:
        out["single_phase"] = single_phase_bench()
    if not args.no_d3q15:
        out["d3q15"] = d3q15_bench()
    if not args.no_paper_workloads:
        out["paper_workloads"] = paper_workloads_bench()
    if not args.no_cpu_baseline:
        model, nproc, usable = host_cpu()
        workers = max(1, min(CPU_WORKERS_MAX, usable))
        v1, dt1, vall, dtall = cpu_baseline(cfg, phi, args.cpu_steps, workers)
        out["cpu_baseline"] = {"value": round(vall, 3), "unit": "MLUPS", "cores": workers, "kind": "oracle",
                               "sample": f"{cfg['nx']}x{cfg['ny']} spinodal {args.variant}: {workers} "
                                         f"independent copies of the FP64 C oracle (one thread each), "
                                         f"{args.cpu_steps} steps each, slowest {dtall:.1f} s",
                               "single_thread": {"value": round(v1, 3), "seconds": round(dt1, 1)},
                               "cpu_model": model, "nproc": nproc, "usable_cpus": usable}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
