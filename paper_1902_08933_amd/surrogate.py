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
# normalization of the network's channels: (field - shift) / scale for phi, u_x, u_y, p. phi is
# mapped from [0, 1] to [-1, 1]; u and p are normalized per state (see normalization()), since
# over a spinodal run their magnitude grows by three orders.
FIELD_SHIFT = (0.5, 0.0, 0.0, 0.0)
FIELD_SCALE = (0.5, 1e-4, 1e-4, 1e-4)
# smallest scales of phi, u and p: a state at rest (u = 0, p uniform) is not blown up
MIN_SCALE = (1e-3, 1e-6, 1e-7)


def normalization(sim, phi_stats=None):
    """(shift, scale) of the network's channels for the current state of a simulation, or None
    when the state is not finite: phi and p shifted by their means and divided by their standard
    deviations, u_x and u_y divided by the larger of their two standard deviations (FP64
    statistics on the GPU, lbpf_field_stats). Over a spinodal run the fluctuations of phi grow
    from 1e-2 to 1/2 and those of u and p by three orders, so every state is brought to unit
    scale. A pair (x_t, x_{t+K}) is normalized with the statistics of x_t. With phi_stats (a
    dict), phi's statistics are also left there."""
    st = sim.field_stats_many(("phi", "ux", "uy", "p"))
    if phi_stats is not None:
        phi_stats.update(st["phi"])
    return _norm_of(st)


_STATE_FIELDS = ("phi", "ux", "uy", "p", "mu")


def _norm_of(st):
    """normalization() from the statistics of phi, ux, uy and p"""
    sphi, sx, sy, sp = st["phi"], st["ux"], st["uy"], st["p"]
    vals = [sphi["mean"], sphi["std"], sx["std"], sy["std"], sp["mean"], sp["std"]]
    if not all(math.isfinite(v) for v in vals):
        return None
    su = max(sx["std"], sy["std"], MIN_SCALE[1])
    return ((sphi["mean"], 0.0, 0.0, sp["mean"]),
            (max(sphi["std"], MIN_SCALE[0]), su, su, max(sp["std"], MIN_SCALE[2])))


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


class TrajectoryStore:
    """Snapshots of solver trajectories every K steps: groups of trajectories, each a tensor of
    raw fields (phi, u_x, u_y, p) as FP32 NHWC [S, T, n, n, 4] on the GPU with the normalization
    of every snapshot; pairs (t, t + K) of one trajectory are drawn from it, both normalized with
    the statistics of the earlier snapshot."""

    def __init__(self, groups):
        import torch
        self.groups = groups  # [(snaps, shift [S, T, 4], scale [S, T, 4])]
        rows = []
        for g, (snaps, shift, _) in enumerate(groups):
            ok = torch.isfinite(shift).all(dim=-1)
            pr = torch.nonzero(ok[:, :-1] & ok[:, 1:], as_tuple=False)
            rows.append(torch.cat([torch.full((pr.shape[0], 1), g, dtype=pr.dtype, device=pr.device), pr], 1))
        self.pairs = torch.cat(rows).cpu().numpy()  # [(group, trajectory, t)]

    @property
    def npairs(self):
        return int(self.pairs.shape[0])

    @property
    def nbytes(self):
        return sum(g[0].numel() * 4 for g in self.groups)

    def batch(self, idx):
        """normalized inputs and targets of the pairs at rows idx of self.pairs (one group)"""
        import torch
        rows = self.pairs[np.asarray(idx)]
        assert (rows[:, 0] == rows[0, 0]).all(), "a batch draws from one group"
        snaps, shift, scale = self.groups[int(rows[0, 0])]
        s = torch.from_numpy(rows[:, 1]).cuda()
        t = torch.from_numpy(rows[:, 2]).cuda()
        sh = shift[s, t][:, None, None, :]
        sc = scale[s, t][:, None, None, :]
        x = ((snaps[s, t] - sh) / sc).contiguous()
        y = ((snaps[s, t + 1] - sh) / sc).contiguous()
        return x, y


def record_trajectories(insts, t_start, t_end, stride=K_STEPS):
    """Runs the instances (cfg, phi0) of one grid size in one batch and records every instance
    from t_start to t_end every `stride` steps: raw fields and their normalization. Snapshots of
    instances that end non-finite get a NaN normalization (their pairs are not drawn)."""
    import torch
    b = lbpf.Batch([c for c, _ in insts])
    for k, (_, phi) in enumerate(insts):
        b.init(k, torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    n_y, n_x = insts[0][1].shape
    T = (t_end - t_start) // stride + 1
    S = len(insts)
    snaps = torch.zeros((S, T, n_y, n_x, 4), dtype=torch.float32, device="cuda")
    shift = np.full((S, T, 4), np.nan, dtype=np.float32)
    scale = np.ones((S, T, 4), dtype=np.float32)
    views = [b.instance(k) for k in range(S)]
    b.step(t_start)
    raw_shift, raw_scale = (0.0, 0.0, 0.0, 0.0), (1.0, 1.0, 1.0, 1.0)
    for j in range(T):
        for k in range(S):
            norm = normalization(views[k])
            if norm is not None:
                lbpf.fields_to_nhwc(views[k], raw_shift, raw_scale, out=snaps[k, j])
                shift[k, j], scale[k, j] = norm
        if j + 1 < T:
            b.step(stride)
    flags, _ = b.status()
    shift[np.asarray(flags, dtype=bool)] = np.nan
    return snaps, torch.from_numpy(shift).cuda(), torch.from_numpy(scale).cuda()


def generate_store(n=256, n_spinodal=256, n_merger=256, spinodal_t=(1000, 11000), merger_t=(0, 5000),
                   stride=K_STEPS, seed=0):
    """Training trajectories of the solver: spinodal runs (the spinodal workload at n x n, seeds
    seed .. seed + n_spinodal - 1) recorded from spinodal_t[0] to spinodal_t[1] and droplet
    mergers from merger_t[0] to merger_t[1], every `stride` steps, each group in one batched
    launch per step."""
    groups = []
    if n_spinodal:
        groups.append(record_trajectories([spinodal_cfg(n, seed + k) for k in range(n_spinodal)],
                                          spinodal_t[0], spinodal_t[1], stride))
    if n_merger:
        groups.append(record_trajectories([merger_cfg(n, seed + k) for k in range(n_merger)],
                                          merger_t[0], merger_t[1], stride))
    return TrajectoryStore(groups)


def train_store(net, store, steps=6000, batch=8, lr=5e-4, seed=0, loss_weights=None, holdout=None,
                log_every=0):
    """Adam on random mini-batches of the store's pairs (those not in `holdout`, a boolean mask
    over the pairs), cosine learning-rate decay; returns the losses."""
    if loss_weights is not None:
        net.set_loss_weights(loss_weights)
    rng = np.random.default_rng(seed)
    pool = np.arange(store.npairs) if holdout is None else np.nonzero(~holdout)[0]
    # batches are drawn from one group at a time, groups in proportion to their pairs
    by_group = [pool[store.pairs[pool, 0] == g] for g in range(len(store.groups))]
    weight = np.array([len(p) for p in by_group], dtype=np.float64)
    weight /= weight.sum()
    losses = []
    for it in range(steps):
        g = rng.choice(len(by_group), p=weight)
        xb, yb = store.batch(rng.choice(by_group[g], size=batch, replace=False))
        a = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        losses.append(net.train_step(xb, yb, a))
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(f"  train step {it}: loss {losses[-1]:.4e}", flush=True)
    return losses


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


def _healthy(sim, max_u, max_phi):
    """finite, |u| <= max_u and |phi| <= max_phi"""
    d = sim.diagnostics(check=False)
    return d["status"] == 0 and d["max_u"] <= max_u and sim.field_stats("phi")["max_abs"] <= max_phi


def hybrid_cycle(sim, net, bufs, ckpt=None, lb_every=500, lb_steps=K_STEPS, max_u=0.1, norm=None,
                 max_growth=10.0, max_phi=1.1, ckpt_prev=None, carry=None):
    """One cycle of the hybrid: (lb_every - lb_steps) / K network strides from the solver's
    current fields, then one LB stride of lb_steps steps re-started from the network's fields
    (equilibrium populations). The cycle ends on an LB state at step + lb_every. The fields are
    normalized with `norm` = (shift, scale), by default the statistics of the current state.

    Fallback: with a checkpoint buffer (lbpf.Simulation.state_size() bytes), the state is saved
    first and restored, and the cycle redone with the plain LB, if the LB stride ends with a
    non-finite state, |u| > max_u, |phi| > max_phi, or a largest |u| or |mu| or a standard
    deviation of phi or u more than max_growth times its value at the cycle's start. A state that
    an earlier cycle left can pass that test and still diverge later: with ckpt_prev (the
    checkpoint saved at the start of the previous cycle, or a list of the checkpoints of the
    previous cycles, newest first), a plain-LB redo that itself ends non-finite or out of range
    is replaced by j + 2 cycles of the plain LB from the checkpoint j cycles further back, for
    j = 0, 1, ... until one ends in range (or the list ends).
    carry (a dict, optional) passes the statistics of a kept cycle's final state to the next
    cycle, which starts from that state and so need not compute them again (each one waits for
    the GPU); it is emptied when the cycle ends with the plain LB.
    Returns True when the network's cycle was kept."""
    a, b = bufs
    step0 = sim.step_count
    have = carry is not None and "u0" in carry
    st0 = None
    if ckpt is not None:
        sim.save_state(out=ckpt)
        if not have:
            st0 = sim.field_stats_many(_STATE_FIELDS)
        u0 = carry["u0"] if have else sim.diagnostics(check=False)["max_u"]
        mu0 = carry["mu0"] if have else st0["mu"]["max_abs"]
    if norm is None:
        norm = carry["norm"] if have else (_norm_of(st0) if st0 is not None else normalization(sim))
    if carry is not None:
        carry.clear()
    if norm is None:  # the state is not finite: nothing for the network to start from
        sim.step(lb_every)
        return False
    shift, scale = norm
    lbpf.fields_to_nhwc(sim, shift, scale, out=a[0])
    strides = (lb_every - lb_steps) // K_STEPS
    for _ in range(strides):
        net.forward(a, out=b)
        a, b = b, a
    lbpf.init_from_nhwc(sim, a[0], shift, scale, step=step0 + strides * K_STEPS)
    sim.step(lb_steps)
    if ckpt is None:
        return True
    d = sim.diagnostics(check=False)
    if d["status"] == 0 and d["max_u"] <= min(max_u, max(max_growth * u0, 1e-4)):
        st1 = sim.field_stats_many(_STATE_FIELDS)
        new, sphi, mu1 = _norm_of(st1), st1["phi"], st1["mu"]["max_abs"]
        if (new is not None and sphi["max_abs"] <= max_phi and new[1][0] <= max_growth * scale[0]
                and new[1][1] <= max_growth * scale[1] and mu1 <= max_growth * max(mu0, 1e-6)):
            if carry is not None:
                carry.update(u0=d["max_u"], mu0=mu1, norm=new)
            return True
    sim.load_state(ckpt)
    sim.step(lb_every)
    older = [] if ckpt_prev is None else (list(ckpt_prev) if isinstance(ckpt_prev, (list, tuple)) else [ckpt_prev])
    for j, ck in enumerate(older):
        if _healthy(sim, max_u, max_phi):
            break
        sim.load_state(ck)
        sim.step((j + 2) * lb_every)
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
    norm = normalization(sim)
    if norm is not None:
        shift, scale = norm
        lbpf.fields_to_nhwc(sim, shift, scale, out=a[0])
        lbpf.init_from_nhwc(sim, a[0], shift, scale, step=sim.step_count)
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


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def horizon_eval(net, cfg, phi0, cycles=20, t0=1000, lb_every=500):
    """The hybrid against the plain LB over `cycles` cycles of lb_every steps from the LB state at
    t0, on the grid of cfg: each cycle, the plain LB, the hybrid (with fallback), the control (plain
    LB with the hybrid's hand-over and no network) and the 2x coarser LB (started from the fine
    state at t0) each advance lb_every steps on their own, and the hybrid, the control and the
    coarse LB are scored against the plain LB: phi relative L2 normalized by ||phi - mean phi||,
    u relative L2, and the ratio of characteristic lengths. Times are wall clock in ms around each
    method's cycle (synchronized)."""
    import torch
    def mk():
        return lbpf.Simulation(cfg).init(torch.from_numpy(np.asarray(phi0, dtype=np.float32)).cuda())
    lb, hy, ctl = mk(), mk(), mk()
    for s_ in (lb, hy, ctl):
        s_.step(t0)
    cc = coarse_params(cfg)
    co = coarse_lb_start(lb, cc)
    co_steps = lb_every // 4
    bufs = hybrid_buffers(hy)
    # a ring of checkpoints: the current cycle's and those of the previous ones, for roll-backs
    depth = 4
    ckpts = [torch.empty(hy.state_size(), dtype=torch.uint8, device=hy.device) for _ in range(depth)]
    co.step(co_steps)  # first-call set-up of the coarse grid's kernels, outside the timing
    co = coarse_lb_start(lb, cc)

    def timed(fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t1) * 1e3

    def host(sim, up=False):
        f = {k: sim.read(k).double().cpu().numpy() for k in ("phi", "ux", "uy")}
        if up:  # coarse grid: back to the fine nodes, velocities in fine lattice units
            f = {"phi": upsample2(f["phi"]), "ux": upsample2(f["ux"]) / 2, "uy": upsample2(f["uy"]) / 2}
        return f

    rows = []
    carry = {}  # statistics of the hybrid's state, from its last kept cycle
    for c in range(cycles):
        _, t_lb = timed(lambda: lb.step(lb_every))
        kept, t_hy = timed(lambda: hybrid_cycle(hy, net, bufs, ckpt=ckpts[c % depth], lb_every=lb_every,
                                                ckpt_prev=[ckpts[(c - k) % depth] for k in range(1, min(c, depth - 1) + 1)],
                                                carry=carry))
        lb_reinit_cycle(ctl, bufs, lb_every=lb_every)
        _, t_co = timed(lambda: co.step(co_steps))
        ref, h, r, cg = host(lb), host(hy), host(ctl), host(co, up=True)
        U = np.stack([ref["ux"], ref["uy"]])
        Lref = domain_length(ref["phi"])

        def score(f):
            return {"phi_rel_l2": float(f"{phi_rel_l2(f['phi'], ref['phi']):.4g}"),
                    "u_rel_l2": float(f"{rel_l2(np.stack([f['ux'], f['uy']]), U):.4g}"),
                    "domain_length_ratio": round(domain_length(f["phi"]) / Lref, 4)}
        rows.append({"cycle": c, "t_end": t0 + (c + 1) * lb_every, "lb_ms": round(t_lb, 2),
                     "hybrid_ms": round(t_hy, 2), "coarse_ms": round(t_co, 2), "network_kept": bool(kept),
                     "hybrid": score(h), "control": score(r), "coarse": score(cg),
                     "domain_length": round(Lref, 2)})
    return rows


def continuous_run(net, cfg, phi0, cycles=20, t0=1000, lb_every=500):
    """The hybrid and the plain LB, each run for `cycles` cycles of lb_every steps from the LB
    state at t0 without stopping between cycles (no per-cycle scoring), each timed as a whole:
    the end-to-end rate of the two. The hybrid keeps its checkpoint ring and fallback, so its
    decisions are those of horizon_eval. Returns the times, the speedup, the cycles kept and the
    final state's phi error and domain-length ratio against the plain LB."""
    import torch
    def mk():
        return lbpf.Simulation(cfg).init(torch.from_numpy(np.asarray(phi0, dtype=np.float32)).cuda())
    lb, hy = mk(), mk()
    for s_ in (lb, hy):
        s_.step(t0)
    bufs = hybrid_buffers(hy)
    depth = 4
    ckpts = [torch.empty(hy.state_size(), dtype=torch.uint8, device=hy.device) for _ in range(depth)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lb.step(cycles * lb_every)
    torch.cuda.synchronize()
    t_lb = (time.perf_counter() - t1) * 1e3
    carry, kept = {}, 0
    t1 = time.perf_counter()
    for c in range(cycles):
        kept += bool(hybrid_cycle(hy, net, bufs, ckpt=ckpts[c % depth], lb_every=lb_every,
                                  ckpt_prev=[ckpts[(c - k) % depth] for k in range(1, min(c, depth - 1) + 1)],
                                  carry=carry))
    torch.cuda.synchronize()
    t_hy = (time.perf_counter() - t1) * 1e3
    ref = lb.read("phi").double().cpu().numpy()
    got = hy.read("phi").double().cpu().numpy()
    return {"lb_ms": round(t_lb, 1), "hybrid_ms": round(t_hy, 1), "speedup": round(t_lb / t_hy, 2),
            "cycles_kept": kept, "phi_rel_l2_end": float(f"{phi_rel_l2(got, ref):.4g}"),
            "domain_length_ratio_end": round(domain_length(got) / domain_length(ref), 4)}


def speedups(rows):
    """Per cycle: raw speedup t(LB) / t(hybrid); and the speedup at equal phi error, against the
    cheapest plain LB whose phi error is at most the hybrid's (the coarse LB when its error is
    not larger, else the fine LB itself, error 0)."""
    out = []
    for r in rows:
        e_h, e_c = r["hybrid"]["phi_rel_l2"], r["coarse"]["phi_rel_l2"]
        if not math.isfinite(e_h):  # the hybrid's state is lost: no error to match
            out.append({"cycle": r["cycle"], "raw": round(r["lb_ms"] / r["hybrid_ms"], 2),
                        "at_equal_phi_error": 0.0, "alternative": "none"})
            continue
        alt = r["coarse_ms"] if e_c <= e_h else r["lb_ms"]
        out.append({"cycle": r["cycle"], "raw": round(r["lb_ms"] / r["hybrid_ms"], 2),
                    "at_equal_phi_error": round(alt / r["hybrid_ms"], 2),
                    "alternative": "coarse" if e_c <= e_h else "fine"})
    return out
