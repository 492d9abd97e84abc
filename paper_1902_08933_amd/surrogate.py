"""Learned surrogate around the LB solver: training data from solver trajectories, training with
the library's own forward/backward/Adam kernels, and the hybrid rollout in which the network
advances the fields K steps at a time and the plain LB step takes over periodically.

All arithmetic runs in the HIP library (solver, field hand-over, network); this module only
sequences calls and moves tensors.
"""
import math
import time

import numpy as np

from . import lbpf, workloads

K_STEPS = 50             # time steps the network advances per application
# normalization of the network's channels: (field - shift) / scale for phi, u_x, u_y, p
FIELD_SHIFT = (0.5, 0.0, 0.0, 0.0)
FIELD_SCALE = (0.5, 1e-4, 1e-4, 1e-4)


def spinodal_cfg(n, seed, variant="qim"):
    return workloads.spinodal(n=n, variant=variant, seed=seed, amplitude=0.005)


def merger_cfg(n, seed):
    """Two droplets of phase A in B, gap of 1..4 nodes between the interfaces, density ratio
    1..10 (seeded): the droplet-merger trajectories of the training set."""
    rng = np.random.default_rng(10_000 + seed)
    r1, r2 = rng.uniform(n / 16, n / 8, size=2)
    gap = rng.uniform(1.0, 4.0)
    ratio = float(rng.uniform(1.0, 10.0))
    cfg, _ = workloads.static_droplet(n=n, R=r1, rho_ratio=ratio, sigma=0.01)
    cfg = dict(cfg, fsurf="mu_grad_phi", name="droplet_merger")
    x1 = n / 2 - (r1 + r2 + gap) / 2
    x2 = x1 + r1 + r2 + gap
    phi = np.maximum(workloads.periodic_droplet_phi(n, n, r1, 4.0, xc=x1, yc=n / 2),
                     workloads.periodic_droplet_phi(n, n, r2, 4.0, xc=x2, yc=n / 2))
    return cfg, phi


def generate_pairs(n=256, n_spinodal=16, n_merger=16, t0=400, snapshots=12, stride=K_STEPS,
                   seed=0):
    """Trajectories of the solver (one batched launch per step over all of them); returns
    normalized NHWC tensors x[t], x[t + stride] on the GPU, shape [pairs, n, n, 4]."""
    import torch
    insts = [spinodal_cfg(n, seed + k) for k in range(n_spinodal)]
    insts += [merger_cfg(n, seed + k) for k in range(n_merger)]
    b = lbpf.Batch([c for c, _ in insts])
    for k, (_, phi) in enumerate(insts):
        b.init(k, torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    b.step(t0)
    snaps = torch.empty((snapshots, len(insts), n, n, 4), dtype=torch.float32, device="cuda")
    for s in range(snapshots):
        for k in range(len(insts)):
            lbpf.fields_to_nhwc(b.instance(k), FIELD_SHIFT, FIELD_SCALE, out=snaps[s, k])
        if s + 1 < snapshots:
            b.step(stride)
    flags, _ = b.status()
    keep = [k for k, f in enumerate(flags) if not f]
    snaps = snaps[:, keep]
    x = snaps[:-1].reshape(-1, n, n, 4).contiguous()
    y = snaps[1:].reshape(-1, n, n, 4).contiguous()
    return x, y


def train(net, x, y, steps=600, batch=4, lr=1e-3, seed=0, log_every=100, loss_weights=None):
    """Adam on random mini-batches of the pairs; cosine learning-rate decay."""
    import torch
    if loss_weights is not None:
        net.set_loss_weights(loss_weights)
    rng = np.random.default_rng(seed)
    m = x.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.from_numpy(rng.choice(m, size=batch, replace=False)).cuda()
        xb = x.index_select(0, idx).contiguous()
        yb = y.index_select(0, idx).contiguous()
        a = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        losses.append(net.train_step(xb, yb, a))
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(f"  train step {it}: loss {losses[-1]:.4e}", flush=True)
    return losses


def eval_one_stride(net, x, y):
    """mean squared error of the network and of persistence (x[t + K] ~ x[t]) on held-out pairs"""
    errs, pers = [], []
    for i in range(x.shape[0]):
        p = net.forward(x[i:i + 1].contiguous())
        errs.append(float(((p - y[i:i + 1]) ** 2).mean()))
        pers.append(float(((x[i:i + 1] - y[i:i + 1]) ** 2).mean()))
    return float(np.mean(errs)), float(np.mean(pers))


def hybrid_cycle(sim, net, bufs, ckpt=None, lb_every=500, lb_steps=K_STEPS, max_u=0.1):
    """One cycle of the hybrid: (lb_every - lb_steps) / K network strides from the solver's
    current fields, then one LB stride of lb_steps steps re-started from the network's fields
    (equilibrium populations). The cycle ends on an LB state at step + lb_every.

    Fallback: with a checkpoint buffer (lbpf.Simulation.state_size() bytes), the state is saved
    first and, if the LB stride ends with a non-finite state or |u| > max_u, restored and the
    cycle is redone with the plain LB. Returns True when the network's cycle was kept."""
    a, b = bufs
    step0 = sim.step_count
    if ckpt is not None:
        sim.save_state(out=ckpt)
    lbpf.fields_to_nhwc(sim, FIELD_SHIFT, FIELD_SCALE, out=a[0])
    strides = (lb_every - lb_steps) // K_STEPS
    for _ in range(strides):
        net.forward(a, out=b)
        a, b = b, a
    lbpf.init_from_nhwc(sim, a[0], FIELD_SHIFT, FIELD_SCALE, step=step0 + strides * K_STEPS)
    sim.step(lb_steps)
    if ckpt is None:
        return True
    d = sim.diagnostics(check=False)
    if d["status"] == 0 and d["max_u"] <= max_u:
        return True
    sim.load_state(ckpt)
    sim.step(lb_every)
    return False


def hybrid_buffers(sim):
    import torch
    return (torch.empty((1, sim.ny, sim.nx, 4), dtype=torch.float32, device=sim.device),
            torch.empty((1, sim.ny, sim.nx, 4), dtype=torch.float32, device=sim.device))


def phi_rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b - b.mean()))


def domain_length(phi):
    """characteristic domain size 2 pi / <k> from the radially averaged structure factor of
    phi - mean(phi) (a statistic of the coarsening state that is not chaotic)"""
    a = np.asarray(phi, dtype=np.float64)
    a = a - a.mean()
    S = np.abs(np.fft.fft2(a)) ** 2
    ky = np.fft.fftfreq(a.shape[0]) * 2 * np.pi
    kx = np.fft.fftfreq(a.shape[1]) * 2 * np.pi
    k = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    S[0, 0] = 0.0
    return float(2 * np.pi * S.sum() / (k * S).sum())


def lb_reinit_cycle(sim, bufs, lb_every=500):
    """control for the hybrid: the plain LB over the cycle, with the same hand-over (fields out,
    equilibrium populations back in) but no network"""
    a, _ = bufs
    sim.step(lb_every - K_STEPS)
    lbpf.fields_to_nhwc(sim, FIELD_SHIFT, FIELD_SCALE, out=a[0])
    lbpf.init_from_nhwc(sim, a[0], FIELD_SHIFT, FIELD_SCALE, step=sim.step_count)
    sim.step(K_STEPS)


def coarse_params(cfg):
    """The same physics on a grid twice as coarse, in diffusive scaling (dx' = 2 dx, dt' = 4 dt):
    nu and tau_h unchanged in lattice units, W' = W/2, sigma' = 2 sigma (sigma ~ rho L^3/T^2),
    M' = M/4 (M beta, the order parameter's diffusivity, invariant), lattice velocity x2,
    pressure x4; 500 fine steps are 125 coarse steps."""
    return dict(cfg, nx=cfg["nx"] // 2, ny=cfg["ny"] // 2, W=cfg["W"] / 2, sigma=2 * cfg["sigma"],
                M_phi=cfg["M_phi"] / 4)


def coarse_lb_start(sim_fine, cfg_coarse):
    """A coarse simulation started from the fine state: fields averaged over 2 x 2 nodes, velocity
    and pressure rescaled (equilibrium populations of those fields)."""
    import torch
    def pool(t):
        return torch.nn.functional.avg_pool2d(t[None, None], 2)[0, 0].contiguous()
    f = {k: sim_fine.read(k) for k in ("phi", "ux", "uy", "p")}
    return lbpf.Simulation(cfg_coarse).init(pool(f["phi"]), 2 * pool(f["ux"]), 2 * pool(f["uy"]),
                                            4 * pool(f["p"]))


def upsample2(c):
    """bilinear, periodic: coarse node j is the mean of fine nodes 2j, 2j+1 (centre 2j + 1/2)"""
    c = np.asarray(c, dtype=np.float64)
    def axis(n):
        pos = (np.arange(2 * n) - 0.5) / 2.0
        j0 = np.floor(pos).astype(int)
        return j0 % n, (j0 + 1) % n, pos - j0
    a0, a1, wa = axis(c.shape[0])
    b0, b1, wb = axis(c.shape[1])
    r = (1 - wa)[:, None] * c[a0] + wa[:, None] * c[a1]
    return (1 - wb)[None, :] * r[:, b0] + wb[None, :] * r[:, b1]
