"""The learned surrogate end to end: trained on trajectories the solver generates (here a reduced
set: 32 spinodal runs and 16 droplet mergers at 256^2), it beats the method without it
(persistence over one stride of 50 steps), the hybrid solver/surrogate cycle is faster than the
plain LB at a stated phi error, and the LB fallback reproduces the plain LB bit for bit."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_1902_08933_amd import lbpf, surrogate as S
    store = S.generate_store(n=256, n_spinodal=32, n_merger=16, spinodal_t=(1000, 6000), merger_t=(200, 2700),
                             seed=300)
    rng = np.random.default_rng(0)
    hold = rng.random(store.npairs) < 0.05
    net = lbpf.UNet(max_batch=8, max_h=256, max_w=256, train=True, seed=1)
    S.train_store(net, store, steps=4000, batch=8, lr=5e-4, loss_weights=[4.0, 1.0, 1.0, 1.0], holdout=hold,
                  log_every=1000)
    return net, store, hold


def test_trained_network_beats_persistence(trained):
    from paper_1902_08933_amd import lbpf
    net, store, hold = trained
    hi = np.nonzero(hold & (store.pairs[:, 0] == 0))[0][:32]
    fresh = lbpf.UNet(max_batch=8, max_h=256, max_w=256, train=False, seed=1)
    e, p, u = np.zeros(4), np.zeros(4), np.zeros(4)
    for i in range(0, len(hi), 8):
        x, y = store.batch(hi[i:i + 8])
        e += ((net.forward(x) - y) ** 2).mean(dim=(0, 1, 2)).double().cpu().numpy()
        p += ((x - y) ** 2).mean(dim=(0, 1, 2)).double().cpu().numpy()
        u += ((fresh.forward(x) - y) ** 2).mean(dim=(0, 1, 2)).double().cpu().numpy()
    print(f"one stride (normalized mse per channel): net {np.round(e, 5)}, persistence {np.round(p, 5)}, "
          f"untrained {np.round(u, 5)}", flush=True)
    assert np.allclose(u, p, rtol=1e-6, atol=1e-12)  # the untrained network predicts no change
    assert e[0] < 0.1 * p[0]
    assert e.sum() < 0.5 * p.sum()


def test_hybrid_faster_than_lb_at_stated_error(trained):
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    net, _, _ = trained
    cfg, phi = W.spinodal(n=1024, seed=99)
    init = torch.from_numpy(phi.astype(np.float32)).cuda()
    lb = lbpf.Simulation(cfg).init(init)
    hy = lbpf.Simulation(cfg).init(init)
    warm = lbpf.Simulation(cfg).init(init)
    big = lbpf.UNet(max_batch=1, max_h=1024, max_w=1024, train=False, seed=1)
    big.set_params(net.get_params())
    bufs = S.hybrid_buffers(hy)
    ckpt = torch.empty(hy.state_size(), dtype=torch.uint8, device="cuda")
    warm.step(1000)
    S.hybrid_cycle(warm, big, bufs, ckpt=ckpt)  # warm-up of both paths on a third simulation
    warm.step(500)
    lb.step(1000)
    hy.step(1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.step(500)
    torch.cuda.synchronize()
    t_lb = time.perf_counter() - t0
    t0 = time.perf_counter()
    kept = S.hybrid_cycle(hy, big, bufs, ckpt=ckpt)
    torch.cuda.synchronize()
    t_hy = time.perf_counter() - t0
    a = hy.read("phi").double().cpu().numpy()
    b = lb.read("phi").double().cpu().numpy()
    err = S.phi_rel_l2(a, b)
    print(f"1024^2 cycle of 500 steps from t = 1000: LB {t_lb * 1e3:.2f} ms, hybrid {t_hy * 1e3:.2f} ms "
          f"(network kept: {kept}); phi rel L2 vs LB {err:.3e}; domain length "
          f"{S.domain_length(a):.2f} vs {S.domain_length(b):.2f}", flush=True)
    assert kept
    assert hy.step_count == lb.step_count
    assert t_hy < t_lb
    assert err < 0.1
    assert abs(S.domain_length(a) / S.domain_length(b) - 1) < 0.02


def test_continuous_run_faster_than_lb(trained):
    # two cycles from t = 1000 run through without stopping, each method timed as a whole
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    net, _, _ = trained
    big = lbpf.UNet(max_batch=1, max_h=1024, max_w=1024, train=False, seed=1)
    big.set_params(net.get_params())
    cfg, phi = W.spinodal(n=1024, seed=99)
    S.continuous_run(big, cfg, phi, cycles=1, t0=0)  # first calls of both paths
    r = S.continuous_run(big, cfg, phi, cycles=2, t0=1000)
    print(f"continuous 2 cycles: {r}", flush=True)
    assert r["cycles_kept"] == 2
    assert r["speedup"] > 1.0
    assert r["phi_rel_l2_end"] < 0.15
    assert abs(r["domain_length_ratio_end"] - 1) < 0.03


def test_fallback_reproduces_plain_lb(trained):
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    net, _, _ = trained
    cfg, phi = W.spinodal(n=256, seed=5)
    a = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    b = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    a.step(800)
    b.step(800)
    ckpt = torch.empty(a.state_size(), dtype=torch.uint8, device="cuda")
    kept = S.hybrid_cycle(a, net, S.hybrid_buffers(a), ckpt=ckpt, max_u=0.0)  # forces the fallback
    assert not kept
    b.step(500)
    assert a.step_count == b.step_count == 1300
    for f in ("phi", "ux", "uy", "p"):
        np.testing.assert_array_equal(a.read(f).cpu().numpy(), b.read(f).cpu().numpy())


def test_fallback_rolls_back_two_cycles(trained):
    # a plain-LB redo that ends out of range (here forced with max_u = 0) is replaced by two
    # cycles of the plain LB from the previous cycle's checkpoint: bit for bit the plain LB
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    net, _, _ = trained
    cfg, phi = W.spinodal(n=256, seed=6)
    a = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    b = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    a.step(800)
    prev, cur = (torch.empty(a.state_size(), dtype=torch.uint8, device="cuda") for _ in range(2))
    a.save_state(out=prev)
    a.step(500)
    kept = S.hybrid_cycle(a, net, S.hybrid_buffers(a), ckpt=cur, ckpt_prev=prev, max_u=0.0)
    assert not kept
    b.step(1800)
    assert a.step_count == b.step_count == 1800
    for f in ("phi", "ux", "uy", "p"):
        np.testing.assert_array_equal(a.read(f).cpu().numpy(), b.read(f).cpu().numpy())


def test_fallback_rolls_back_further(trained):
    # with the checkpoints of the two previous cycles (newest first) and every state out of range
    # (max_u = 0), the redo goes back two cycles, then three: bit for bit the plain LB
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S, workloads as W
    net, _, _ = trained
    cfg, phi = W.spinodal(n=256, seed=7)
    a = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    b = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    a.step(300)
    old, prev, cur = (torch.empty(a.state_size(), dtype=torch.uint8, device="cuda") for _ in range(3))
    a.save_state(out=old)
    a.step(500)
    a.save_state(out=prev)
    a.step(500)
    kept = S.hybrid_cycle(a, net, S.hybrid_buffers(a), ckpt=cur, ckpt_prev=[prev, old], max_u=0.0)
    assert not kept
    b.step(1800)
    assert a.step_count == b.step_count == 1800
    for f in ("phi", "ux", "uy", "p"):
        np.testing.assert_array_equal(a.read(f).cpu().numpy(), b.read(f).cpu().numpy())


def test_field_stats_many_equals_single_calls():
    # lbpf_field_stats_many: bit for bit the statistics of one lbpf_field_stats call per field,
    # in any order and with repeats
    import torch
    from paper_1902_08933_amd import lbpf, workloads as W
    cfg, phi = W.spinodal(n=192, seed=9, amplitude=0.05)
    sim = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    sim.step(200)
    names = ("mu", "phi", "p", "ux", "uy", "rho")
    many = sim.field_stats_many(names)
    for f in names:
        assert many[f] == sim.field_stats(f), f
    assert sim.field_stats_many(("uy",)) == {"uy": sim.field_stats("uy")}


def test_field_stats_against_host():
    # lbpf_field_stats (FP64 on the GPU) against the same statistics of the read fields
    import torch
    from paper_1902_08933_amd import lbpf, workloads as W
    cfg, phi = W.spinodal(n=200, seed=8, amplitude=0.05)
    sim = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    sim.step(300)
    for f in ("phi", "ux", "uy", "p", "rho", "mu"):
        v = sim.read(f).double().cpu().numpy()
        s = sim.field_stats(f)
        assert abs(s["mean"] - v.mean()) <= 1e-12 * max(1.0, abs(v.mean())) + 1e-15, f
        assert abs(s["std"] - v.std()) <= 1e-9 * v.std() + 1e-15, f
        assert s["max_abs"] == np.abs(v).max(), f
