"""Parity of the HIP solver (FP32 arithmetic, h_0 as an FP32 hi/lo pair) with the FP64 CPU
oracle on the same seeded inputs, through the C ABI: every field is compared over all its
nodes, by relative L2 and by the largest element-wise difference.

Tolerances: relative L2 <= 1e-5 on phi and on u = (u_x, u_y) after 100 steps, and relative
drift of sum(phi) <= 1e-6. The pressure has no stated bound; it is held to 1e-4 (its FP32
error is of the same order as that of u, amplified by the 1/(1 - w_0) of eq. 28). Element-wise
bounds: tests/parity.py.
"""
import numpy as np
import pytest

import oracle
from paper_1902_08933_amd import workloads as W

from parity import MAX_P, MAX_PHI, MAX_U, TOL_DRIFT, TOL_P, TOL_PHI, TOL_U, check

pytestmark = pytest.mark.gpu


def gpu_sim(cfg, phi, tile=None):
    import torch
    from paper_1902_08933_amd import lbpf
    sim = lbpf.Simulation(cfg)
    if tile is not None:
        sim.set_tile(tile)
    sim.init(torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    return sim


def gpu_fields(sim, names=("phi", "ux", "uy", "p", "rho", "mu")):
    return {f: sim.read(f).double().cpu().numpy() for f in names}


def oracle_fields(o, names=("phi", "ux", "uy", "p", "rho", "mu")):
    return {f: o.read(f) for f in names}


def ragged_spinodal(nx, ny, variant, seed=7, **kw):
    cfg, _ = W.spinodal(n=nx, variant=variant, seed=seed, **kw)
    cfg = dict(cfg, nx=nx, ny=ny)
    phi = W.spinodal_phi(nx, ny, 0.5, 0.005, seed)
    return cfg, phi


def small_bubble(variant="qim", rho_ratio=10.0):
    # density ratio 10: from ratio ~50 up the method itself diverges (the FP64 oracle too)
    cfg, _ = W.rising_bubble(nx=96, ny=160, R=16.0, variant=variant, rho_ratio=rho_ratio)
    phi = W.droplet_phi(96, 160, 16.0, 4.0, xc=48.0, yc=64.0, inside=0.0)
    return cfg, phi


def case(name):
    if name == "droplet64_qim":
        return W.static_droplet(n=64, R=16.0, variant="qim")
    if name == "droplet64_im":
        return W.static_droplet(n=64, R=16.0, variant="im")
    if name == "spinodal_100x90_qim":
        return ragged_spinodal(100, 90, "qim")
    if name == "spinodal_100x90_im":
        return ragged_spinodal(100, 90, "im")
    if name == "spinodal_100x90_paper_g0":
        c, p = ragged_spinodal(100, 90, "qim")
        return dict(c, pscheme="eq28_paper_g0"), p
    if name == "spinodal_100x90_eq29":
        c, p = ragged_spinodal(100, 90, "qim")
        return dict(c, pscheme="eq29"), p
    if name == "poiseuille_256x128_qim":
        return W.layered_poiseuille(nx=256, ny=128, mu_ratio=10.0, G=1e-6, variant="qim")
    if name == "poiseuille_256x128_step_visc":
        return W.layered_poiseuille(nx=256, ny=128, mu_ratio=3.0, rho_ratio=3.0, G=1e-6,
                                    visc="step", variant="qim")
    if name == "bubble_96x160_ratio10":
        return small_bubble()
    if name == "droplet_mu_grad_phi_gravity":
        c, p = W.static_droplet(n=48, R=12.0, variant="qim", rho_ratio=5.0)
        return dict(c, fsurf="mu_grad_phi", gravity=2e-6, force_x=1e-6), p
    raise KeyError(name)


CASES = ["droplet64_qim", "droplet64_im", "spinodal_100x90_qim", "spinodal_100x90_im",
         "spinodal_100x90_paper_g0", "spinodal_100x90_eq29", "poiseuille_256x128_qim",
         "poiseuille_256x128_step_visc", "bubble_96x160_ratio10",
         "droplet_mu_grad_phi_gravity"]


@pytest.mark.parametrize("name", CASES)
def test_parity_100_steps(name):
    cfg, phi = case(name)
    phi32 = np.ascontiguousarray(phi, dtype=np.float32)
    print(f"case {name}: {cfg['nx']}x{cfg['ny']} {cfg['variant']} {cfg.get('pscheme')}", flush=True)
    sim = gpu_sim(cfg, phi32)
    d0 = sim.diagnostics()
    sim.step(100)
    g = gpu_fields(sim)
    d1 = sim.diagnostics()
    o = oracle.Oracle(cfg).init(phi32.astype(np.float64)).step(100)
    r = oracle_fields(o)
    check("phi", g["phi"], r["phi"], TOL_PHI, MAX_PHI)
    check("u", np.stack([g["ux"], g["uy"]]), np.stack([r["ux"], r["uy"]]), TOL_U, MAX_U)
    check("p", g["p"], r["p"], TOL_P, MAX_P)
    check("rho", g["rho"], r["rho"], TOL_PHI, MAX_PHI)
    drift = abs(d1["sum_phi"] - d0["sum_phi"]) / abs(d0["sum_phi"])
    print(f"  drift {drift:.2e}", flush=True)
    assert drift <= TOL_DRIFT
    assert abs(d1["sum_phi"] - o.sum_phi()) / abs(o.sum_phi()) <= TOL_DRIFT
    assert d1["nonfinite"] == 0


def test_init_state_matches_oracle():
    cfg, phi = ragged_spinodal(70, 37, "qim", amplitude=0.05)
    phi32 = phi.astype(np.float32)
    g = gpu_fields(gpu_sim(cfg, phi32))
    r = oracle_fields(oracle.Oracle(cfg).init(phi32.astype(np.float64)))
    check("phi", g["phi"], r["phi"], 1e-7, 1e-7)
    check("mu", g["mu"], r["mu"], 1e-5, 1e-4)
    check("u", np.stack([g["ux"], g["uy"]]), np.stack([r["ux"], r["uy"]]), 1e-5, MAX_U)


@pytest.mark.parametrize("nx,ny,bc", [(3, 3, "periodic"), (3, 5, "walls_y"), (65, 17, "walls_y"),
                                      (130, 3, "periodic"), (5, 200, "walls_y")])
def test_parity_edge_grids(nx, ny, bc):
    cfg, _ = W.spinodal(n=nx, variant="qim", seed=11)
    cfg = dict(cfg, nx=nx, ny=ny, bc=bc, force_x=1e-6)
    phi = W.spinodal_phi(nx, ny, 0.5, 0.05, 11).astype(np.float32)
    print(f"edge grid {nx}x{ny} {bc}", flush=True)
    sim = gpu_sim(cfg, phi)
    sim.step(50)
    g = gpu_fields(sim)
    r = oracle_fields(oracle.Oracle(cfg).init(phi.astype(np.float64)).step(50))
    check("phi", g["phi"], r["phi"], TOL_PHI, MAX_PHI)
    check("u", np.stack([g["ux"], g["uy"]]), np.stack([r["ux"], r["uy"]]), TOL_U, MAX_U)


def test_zero_steps_is_noop():
    cfg, phi = W.static_droplet(n=32, R=8.0)
    sim = gpu_sim(cfg, phi)
    a = gpu_fields(sim)
    sim.step(0)
    b = gpu_fields(sim)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    assert sim.step_count == 0


def test_tile_shapes_bit_identical():
    from paper_1902_08933_amd import lbpf
    cfg, phi = ragged_spinodal(150, 70, "qim", amplitude=0.05)
    ref = None
    for t in range(len(lbpf.tile_shapes())):
        print(f"tile {t} {lbpf.tile_shapes()[t]}", flush=True)
        sim = gpu_sim(cfg, phi, tile=t)
        sim.step(30)
        g = gpu_fields(sim, ("phi", "ux", "uy", "p"))
        if ref is None:
            ref = g
        else:
            for k in g:
                np.testing.assert_array_equal(g[k], ref[k])


def test_run_to_run_deterministic():
    cfg, phi = ragged_spinodal(128, 64, "qim", amplitude=0.05)
    runs = []
    for _ in range(2):
        sim = gpu_sim(cfg, phi)
        sim.step(40)
        runs.append((gpu_fields(sim, ("phi", "ux", "uy", "p")), sim.diagnostics()))
    for k in runs[0][0]:
        np.testing.assert_array_equal(runs[0][0][k], runs[1][0][k])
    assert runs[0][1]["sum_phi"] == runs[1][1]["sum_phi"]


def test_checkpoint_resume_bitwise():
    cfg, phi = small_bubble()
    a = gpu_sim(cfg, phi)
    a.step(40)
    b = gpu_sim(cfg, phi)
    b.step(20)
    buf = b.save_state()
    c = gpu_sim(cfg, np.zeros_like(phi))
    c.load_state(buf)
    assert c.step_count == 20
    c.step(20)
    ga, gc = gpu_fields(a), gpu_fields(c)
    for k in ga:
        np.testing.assert_array_equal(ga[k], gc[k])


def test_diagnostics_against_oracle():
    cfg, phi = W.static_droplet(n=64, R=16.0)
    phi32 = phi.astype(np.float32)
    sim = gpu_sim(cfg, phi32)
    sim.step(200)
    d = sim.diagnostics()
    o = oracle.Oracle(cfg).init(phi32.astype(np.float64)).step(200)
    rho = o.read("rho")
    umax = np.hypot(o.read("ux"), o.read("uy")).max()
    assert abs(d["sum_phi"] - o.sum_phi()) / o.sum_phi() < 1e-7
    assert abs(d["sum_rho"] - rho.sum()) / rho.sum() < 1e-7
    assert abs(d["max_u"] - umax) / umax < 1e-4
    assert d["step"] == 200 and d["nonfinite"] == 0


def test_laplace_dp_against_oracle():
    cfg, phi = W.static_droplet(n=64, R=16.0)
    phi32 = phi.astype(np.float32)
    sim = gpu_sim(cfg, phi32)
    sim.step(300)
    dp_gpu = sim.laplace_dp(32.0, 32.0, 16.0)
    o = oracle.Oracle(cfg).init(phi32.astype(np.float64)).step(300)
    P = o.laplace_pressure()
    x = np.arange(64)[None, :] - 32.0
    y = np.arange(64)[:, None] - 32.0
    r = np.hypot(np.minimum(abs(x), 64 - abs(x)), np.minimum(abs(y), 64 - abs(y)))
    dp_ref = P[r <= 8.0].mean() - P[r >= 16.0 + 12.0].mean()
    assert abs(dp_gpu - dp_ref) / abs(dp_ref) < 1e-4


def test_nonfinite_state_reported():
    from paper_1902_08933_amd import lbpf
    cfg, phi = W.static_droplet(n=32, R=8.0)
    phi = phi.astype(np.float32)
    phi[5, 7] = np.nan
    sim = gpu_sim(cfg, phi)
    sim.step(3)
    d = sim.diagnostics(check=False)
    assert d["status"] == -4 and d["nonfinite"] > 0
    with pytest.raises(lbpf.LbpfError):
        sim.diagnostics()


@pytest.mark.parametrize("variant", ["qim", "im"])
def test_full_size_spinodal_1024(variant):
    # the 1024 x 1024 spinodal workload at the launch configuration the benchmark times:
    # full-field parity after 5 steps, and conservation over 2000 steps
    cfg, phi = W.spinodal(n=1024, variant=variant, seed=0)
    phi32 = phi.astype(np.float32)
    print(f"full size 1024x1024 {variant}", flush=True)
    sim = gpu_sim(cfg, phi32)
    sim.autotune(trial_steps=5)  # the benchmark's strip shape; the state is restored
    assert sim.step_count == 0
    print(f"autotuned strip shape {sim.tile}", flush=True)
    d0 = sim.diagnostics()
    sim.step(5)
    g = gpu_fields(sim, ("phi", "ux", "uy"))
    o = oracle.Oracle(cfg).init(phi32.astype(np.float64)).step(5)
    check("phi", g["phi"], o.read("phi"), TOL_PHI, MAX_PHI)
    check("u", np.stack([g["ux"], g["uy"]]), np.stack([o.read("ux"), o.read("uy")]), TOL_U, MAX_U)
    sim.step(1995)
    d1 = sim.diagnostics()
    assert abs(d1["sum_phi"] - d0["sum_phi"]) / d0["sum_phi"] <= TOL_DRIFT


def test_autotune_restores_state_bitwise():
    from paper_1902_08933_amd import lbpf
    cfg, phi = ragged_spinodal(200, 120, "qim", amplitude=0.05)
    a = gpu_sim(cfg, phi)
    a.step(20)
    best, ms = a.autotune(trial_steps=3)
    assert 0 <= best < len(lbpf.tile_shapes()) and a.tile == best
    assert len(ms) == len(lbpf.tile_shapes()) and all(t > 0 for t in ms)
    assert a.step_count == 20
    a.step(20)
    b = gpu_sim(cfg, phi)
    b.step(40)
    ga, gb = gpu_fields(a), gpu_fields(b)
    for k in ga:
        np.testing.assert_array_equal(ga[k], gb[k])


@pytest.mark.parametrize("walls", [False, True])
def test_state_layouts_bit_identical(walls, monkeypatch):
    # population copies with rows interleaved (the default) and with separate planes hold the same
    # values at other addresses: every field after 30 steps is bitwise equal, and a checkpoint of
    # one layout is refused by a simulation of the other
    import torch
    from paper_1902_08933_amd import lbpf
    cfg, phi = ragged_spinodal(70, 33, "qim")
    if walls:
        cfg = dict(cfg, bc="walls_y", force_x=1e-5, gravity=2e-6)
    out, diag, sims = {}, {}, {}
    for layout in ("interleaved", "planar"):
        if layout == "planar":
            monkeypatch.setenv("LBPF_STATE_LAYOUT", "planar")
        sim = gpu_sim(cfg, phi)
        sim.step(30)
        out[layout] = gpu_fields(sim)
        diag[layout] = sim.diagnostics()
        sims[layout] = sim
    for k in out["interleaved"]:
        assert np.array_equal(out["interleaved"][k], out["planar"][k]), k
    assert diag["interleaved"] == diag["planar"]
    ckpt = sims["interleaved"].save_state()
    buf = torch.zeros(max(ckpt.numel(), sims["planar"].state_size()), dtype=torch.uint8, device="cuda")
    buf[:ckpt.numel()] = ckpt
    with pytest.raises(lbpf.LbpfError):
        sims["planar"].load_state(buf)  # the header names the other layout


def test_large_grid_separate_planes_against_oracle_crop():
    # 8192 x 6400 nodes: a population copy interleaved by row would need per-lane offsets of
    # 2^30 floats or more, so this grid keeps separate planes (the workspace size says which);
    # two steps from a seeded spinodal field, then the inner 20^2 nodes of a 40^2 periodic crop
    # around the grid corner against the oracle run on that crop (the fields read after two
    # steps depend on the initial field within a radius of 9 nodes)
    from paper_1902_08933_amd import lbpf
    nx, ny = 8192, 6400
    cfg, _ = W.spinodal(n=64, variant="qim", seed=3)
    cfg = dict(cfg, nx=nx, ny=ny)
    xp, pad, red = nx, 4160, (4096 * 8 + 64) * 8
    assert lbpf.workspace_size(cfg) == (2 * 21 * (ny * xp + pad) + 2 * ny * xp) * 4 + red
    phi = W.spinodal_phi(nx, ny, 0.5, 0.05, 3).astype(np.float32)
    print(f"large grid {nx}x{ny}, separate planes", flush=True)
    sim = gpu_sim(cfg, phi)
    sim.step(2)
    ix, iy = np.arange(-20, 20) % nx, np.arange(-20, 20) % ny
    crop = phi[np.ix_(iy, ix)].astype(np.float64)
    o = oracle.Oracle(dict(cfg, nx=40, ny=40)).init(crop).step(2)
    inner = np.arange(10, 30)
    sel = np.ix_(iy[inner], ix[inner])
    for f, tol, tmax in (("phi", TOL_PHI, MAX_PHI), ("ux", TOL_U, MAX_U), ("uy", TOL_U, MAX_U),
                         ("p", TOL_P, MAX_P)):
        g = sim.read(f)[torch_index(sel)].double().cpu().numpy()
        check(f, g, o.read(f)[np.ix_(inner, inner)], tol, tmax)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0


def torch_index(sel):
    import torch
    return tuple(torch.from_numpy(np.asarray(s)).cuda() for s in sel)


def test_library_opened_before_torch_shares_its_hip_runtime():
    # a fresh interpreter that opens the library (workspace_size) before importing torch itself:
    # the binding imports torch first, so one HIP runtime serves both and the step runs
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import numpy as np\n"
        "from paper_1902_08933_amd import lbpf, workloads as W\n"
        "cfg, phi = W.static_droplet(n=32, R=8.0)\n"
        "lbpf.workspace_size(cfg)\n"
        "import torch\n"
        "sim = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())\n"
        "sim.step(3)\n"
        "print('steps', sim.diagnostics()['step'])\n"
    )
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "steps 3" in r.stdout


@pytest.mark.parametrize("tile", [15, None])
def test_bench_4096_interleaved_against_oracle_crop(tile):
    # the benchmark's 4096^2 spinodal: rows longer than 4 KiB, so the 21 planes of a copy are
    # interleaved by row with no pad between them (the workspace size says which layout), at strip
    # shape 15 (256 x 32, 512 threads: the one the autotuner picks there) and at the shape the
    # autotuner picks on this machine; two steps, then the inner 20^2 nodes of a 40^2 periodic crop
    # around the grid corner against the oracle run on that crop
    from paper_1902_08933_amd import lbpf
    n = 4096
    cfg, phi = W.spinodal(n=n, variant="qim", seed=0)
    red = (4096 * 8 + 64) * 8
    assert lbpf.workspace_size(cfg) == (2 * (21 * n * n + 4160) + 2 * n * n) * 4 + red
    phi32 = phi.astype(np.float32)
    sim = gpu_sim(cfg, phi32, tile=tile)
    if tile is None:
        sim.autotune(trial_steps=3)
        assert sim.step_count == 0
    print(f"4096^2 interleaved, strip shape {sim.tile} {lbpf.tile_shapes()[sim.tile]}", flush=True)
    sim.step(2)
    ix = np.arange(-20, 20) % n
    crop = phi32[np.ix_(ix, ix)].astype(np.float64)
    o = oracle.Oracle(dict(cfg, nx=40, ny=40)).init(crop).step(2)
    inner = np.arange(10, 30)
    sel = np.ix_(ix[inner], ix[inner])
    for f, tol, tmax in (("phi", TOL_PHI, MAX_PHI), ("ux", TOL_U, MAX_U), ("uy", TOL_U, MAX_U),
                         ("p", TOL_P, MAX_P)):
        g = sim.read(f)[torch_index(sel)].double().cpu().numpy()
        check(f, g, o.read(f)[np.ix_(inner, inner)], tol, tmax)
    # and a crop in the middle of the grid, away from every periodic seam
    c0 = n // 2 - 20
    jx = np.arange(c0, c0 + 40)
    o = oracle.Oracle(dict(cfg, nx=40, ny=40)).init(phi32[np.ix_(jx, jx)].astype(np.float64)).step(2)
    sel = np.ix_(jx[inner], jx[inner])
    for f, tol, tmax in (("phi", TOL_PHI, MAX_PHI), ("ux", TOL_U, MAX_U), ("uy", TOL_U, MAX_U)):
        g = sim.read(f)[torch_index(sel)].double().cpu().numpy()
        check(f, g, o.read(f)[np.ix_(inner, inner)], tol, tmax)
    assert sim.diagnostics()["nonfinite"] == 0
