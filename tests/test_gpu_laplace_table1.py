"""Laplace's law at density ratio 50 (Sec. 4.2, Table 1) on the HIP D2Q9 solver: the printed
setup (100 x 100 periodic, droplet of radius R = 20 ... 40 centred at (50, 50) with the eq. (36)
profile, F_s = -phi grad mu, rho_B = 1, tau_h = 1, tau_g = 0.8, sigma = 0.001, M_phi = 0.02,
W = 4), run to t = 5 x 10^5 as in the paper; the relative error of the pressure jump against
sigma / R is compared with the printed one for both variants.

Measured: QIM 0.07 / 0.34 / 0.48 / 0.54 / 0.54 % and IM 0.32 / 0.72 / 0.90 / 0.99 / 1.07 % for
R = 20 ... 40, against the printed 0.02 / 0.45 / 0.42 / 0.53 / 0.68 % and 0.36 / 0.73 / 0.84 /
0.95 / 1.00 %; every case lies within 0.15 percentage points of the paper's value, all below
sigma / R. The test allows 0.25 points. The FP64 oracle cannot afford 5 x 10^5 steps on 100^2
here, so the GPU is tied to it in the same regime by element-wise parity over 100 steps.
"""
import numpy as np
import pytest

import oracle
from paper_1902_08933_amd import workloads as W
from parity import MAX_P, MAX_PHI, MAX_U, check
from test_oracle_physics import load_golden

pytestmark = pytest.mark.gpu

TABLE1 = load_golden("table1_laplace.txt")  # R, error QIM, error IM


def droplet50(R, variant):
    return W.static_droplet(n=100, R=R, variant=variant, rho_ratio=50.0, sigma=0.001, tau=0.8,
                            tau_h=1.0, M_phi=0.02, W=4.0)


def gpu_sim(cfg, phi):
    import torch
    from paper_1902_08933_amd import lbpf
    sim = lbpf.Simulation(cfg)
    sim.init(torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    return sim


@pytest.mark.parametrize("variant", ["qim", "im"])
@pytest.mark.parametrize("R", [20.0, 25.0, 30.0, 35.0, 40.0])
def test_table1_pressure_jump(R, variant):
    row = TABLE1[TABLE1[:, 0] == R][0]
    printed = row[1] if variant == "qim" else row[2]
    cfg, phi = droplet50(R, variant)
    print(f"table 1 {variant} R {R:g}: 5e5 steps", flush=True)
    sim = gpu_sim(cfg, phi)
    sim.step(500000)
    d = sim.diagnostics()
    err = sim.laplace_dp(50.0, 50.0, R) / (cfg["sigma"] / R) - 1.0
    print(f"  error {err:+.4%} (printed {printed:.2%}), max|u| {d['max_u']:.1e}", flush=True)
    assert d["nonfinite"] == 0
    assert abs(abs(err) - printed) <= 0.0025


@pytest.mark.parametrize("variant", ["qim", "im"])
def test_density_ratio_50_parity(variant):
    # element-wise against the FP64 oracle after 100 steps, R = 25, same bars as the other
    # parity cases (phi, u 1e-5; p 1e-4), and the pressure jump of the two within 1e-4
    cfg, phi = droplet50(25.0, variant)
    phi = phi.astype(np.float32).astype(np.float64)
    o = oracle.Oracle(cfg).init(phi).step(100)
    sim = gpu_sim(cfg, phi)
    sim.step(100)

    g = {f: sim.read(f).double().cpu().numpy() for f in ("phi", "ux", "uy", "p")}
    e_phi, _ = check("phi", g["phi"], o.read("phi"), 1e-5, MAX_PHI)
    e_u, _ = check("u", np.stack([g["ux"], g["uy"]]), np.stack([o.read("ux"), o.read("uy")]), 1e-5, MAX_U)
    e_p, _ = check("p", g["p"], o.read("p"), 1e-4, MAX_P)
    P = o.laplace_pressure()
    x = np.arange(100)[None, :] - 50.0
    y = np.arange(100)[:, None] - 50.0
    r = np.hypot(np.minimum(abs(x), 100 - abs(x)), np.minimum(abs(y), 100 - abs(y)))
    dp_ref = P[r <= 12.5].mean() - P[r >= 25.0 + 12.0].mean()
    dp = sim.laplace_dp(50.0, 50.0, 25.0)
    print(f"  phi {e_phi:.2e} u {e_u:.2e} p {e_p:.2e} dP {abs(dp / dp_ref - 1):.2e}", flush=True)
    assert e_phi <= 1e-5 and e_u <= 1e-5 and e_p <= 1e-4
    assert abs(dp - dp_ref) <= 1e-4 * abs(dp_ref)
