"""The learned surrogate end to end: trained on trajectories the solver generates, it beats the
method without it (persistence over one stride of 50 steps), the hybrid solver/surrogate cycle
is faster than the plain LB at a stated phi error, and the LB fallback reproduces the plain LB
bit for bit."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    from paper_1902_08933_amd import lbpf, surrogate as S
    xs, ys = S.generate_pairs(n=256, n_spinodal=24, n_merger=4, t0=1000, snapshots=16, seed=3)
    perm = torch.from_numpy(np.random.default_rng(0).permutation(xs.shape[0])).cuda()
    xs, ys = xs[perm].contiguous(), ys[perm].contiguous()
    ntr = int(xs.shape[0] * 0.85)
    net = lbpf.UNet(max_batch=8, max_h=256, max_w=256, train=True, seed=1)
    S.train(net, xs[:ntr], ys[:ntr], steps=2000, batch=8, lr=5e-4, log_every=500,
            loss_weights=[400.0, 1.0, 1.0, 1.0])
    return net, xs[ntr:], ys[ntr:]


def test_trained_network_beats_persistence(trained):
    from paper_1902_08933_amd import lbpf, surrogate as S
    net, xv, yv = trained
    e_all, p_all = S.eval_one_stride(net, xv, yv)
    k = min(8, xv.shape[0])
    e_phi = float(((net.forward(xv[:k].contiguous())[..., 0] - yv[:k, ..., 0]) ** 2).mean())
    p_phi = float(((xv[:k, ..., 0] - yv[:k, ..., 0]) ** 2).mean())
    fresh = lbpf.UNet(max_batch=8, max_h=256, max_w=256, train=False, seed=1)
    u_all, _ = S.eval_one_stride(fresh, xv, yv)
    print(f"one stride: net {e_all:.3e} / phi {e_phi:.3e}; persistence {p_all:.3e} / phi {p_phi:.3e}; "
          f"untrained {u_all:.3e}", flush=True)
    assert abs(u_all - p_all) <= 1e-6 * p_all + 1e-12  # the untrained network predicts no change
    assert e_phi < 0.1 * p_phi
    assert e_all < 0.5 * p_all


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
    print(f"1024^2 cycle of 500 steps: LB {t_lb * 1e3:.2f} ms, hybrid {t_hy * 1e3:.2f} ms "
          f"(network kept: {kept}); phi rel L2 vs LB {err:.3e}; domain length "
          f"{S.domain_length(a):.2f} vs {S.domain_length(b):.2f}", flush=True)
    assert kept
    assert hy.step_count == lb.step_count
    assert t_hy < t_lb
    assert err < 0.15
    assert abs(S.domain_length(a) / S.domain_length(b) - 1) < 0.02


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
