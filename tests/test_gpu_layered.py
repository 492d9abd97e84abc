"""Layered Poiseuille flow (Sec. 4.3) on the HIP solvers, D2Q9 and D3Q15, at the printed channel
height NY = 100 and the four viscosity ratios of Table 2: the steady velocity against eq. (37)
with the printed error norm, bounded by the error Table 2 reports for the paper's own models.

Only the ratio mu_A/mu_B is printed, not the two viscosities. Under BGK the slip of halfway
bounce-back grows with the relaxation time, so holding nu_B = 0.1 puts the upper fluid at
tau = 30.5 (ratio 100) and 300.5 (ratio 1000), where the wall slip alone exceeds the printed
error (3.0 % and 24.6 % in the FP64 oracle, almost all of it in the upper half). These cases hold
the geometric mean of the two kinematic viscosities at 0.1 instead and run
max(150000, 1.2 h^2 / nu_B) steps, past the point where the error stops changing: the FP64
oracle (D2Q9) gives 0.074 %, 0.263 %, 0.668 % and 0.765 % there, unchanged to 0.01 % with half
as many steps again. The GPU's FP32 rounding moves these by up to 0.15 % either way (near
tau = 1/2 the flow keeps a memory of ~10^5 steps). The channel is x-invariant, so four columns
(4 x 4 in three dimensions) stand in for the printed NX = 10.
"""
import time

import numpy as np
import pytest

from paper_1902_08933_amd import workloads as W

from analytic import layered_analytic_ux

pytestmark = pytest.mark.gpu

NY = 100
TABLE2 = {3.0: 0.0104, 10.0: 0.0130, 100.0: 0.0190, 1000.0: 0.0216}


def setup(ratio):
    h = NY / 2.0
    nu_A, nu_B = W.table2_viscosities(ratio)
    G = 5e-5 * (nu_A + nu_B) / h ** 2  # u_c (mu_A + mu_B) / h^2 at unit density
    steps = max(150000, int(1.2 * h * h / nu_B))
    return nu_B, G, steps, layered_analytic_ux(NY, G, nu_A, nu_B)


def error(u, ua):
    return float(np.abs(u - ua).sum() / np.abs(ua).sum())


@pytest.mark.parametrize("ratio", sorted(TABLE2))
def test_layered_poiseuille_d2q9(ratio):
    import torch
    from paper_1902_08933_amd import lbpf
    nu_B, G, steps, ua = setup(ratio)
    cfg, phi = W.layered_poiseuille(nx=4, ny=NY, mu_ratio=ratio, nu_B=nu_B, G=G)
    print(f"layered d2q9 ratio {ratio:g}: {steps} steps", flush=True)
    sim = lbpf.Simulation(cfg)
    sim.init(torch.from_numpy(phi.astype(np.float32)).cuda())
    t = time.time()
    sim.step(steps)
    u = sim.read("ux").double().cpu().numpy()
    e = error(u[:, 0], ua)
    print(f"  error {e:.4%} (Table 2: {TABLE2[ratio]:.2%}), {time.time() - t:.1f} s", flush=True)
    assert np.allclose(u, u[:, :1], rtol=0, atol=1e-12 + 1e-6 * np.abs(ua).max())
    assert e <= TABLE2[ratio]


@pytest.mark.parametrize("ratio", sorted(TABLE2))
def test_layered_poiseuille_d3q15(ratio):
    import torch
    from paper_1902_08933_amd import lbpf
    nu_B, G, steps, ua = setup(ratio)
    cfg, phi = W.layered_poiseuille3d(nxy=4, nz=NY, mu_ratio=ratio, nu_B=nu_B, G=G)
    print(f"layered d3q15 ratio {ratio:g}: {steps} steps", flush=True)
    sim = lbpf.Simulation3D(cfg)
    shapes = lbpf.shapes3d()  # (tile x, tile y, z chunk)
    sim.set_shape(min(range(len(shapes)), key=lambda s: shapes[s][2]))  # most workgroups on 100 planes
    sim.init(torch.from_numpy(phi.astype(np.float32)).cuda())
    t = time.time()
    sim.step(steps)
    u = sim.read("ux").double().cpu().numpy()
    e = error(u[:, 0, 0], ua)
    print(f"  error {e:.4%} (Table 2: {TABLE2[ratio]:.2%}), {time.time() - t:.1f} s", flush=True)
    assert np.allclose(u, u[:, :1, :1], rtol=0, atol=1e-12 + 1e-6 * np.abs(ua).max())
    assert np.abs(sim.read("uy").double().cpu().numpy()).max() < 1e-6 * np.abs(ua).max()
    assert e <= TABLE2[ratio]
