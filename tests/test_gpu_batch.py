"""Batched persistent launch: every instance evolves bit-identically to a single simulation,
graph replays equal single launches, diverged instances are frozen without disturbing the
others, and one instance is checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1902_08933_amd import workloads as W

pytestmark = pytest.mark.gpu


def mixed_instances():
    out = []
    c, p = W.static_droplet(n=48, R=12.0, variant="qim")
    out.append((c, p))
    c, p = W.layered_poiseuille(nx=70, ny=33, mu_ratio=10.0, G=1e-5, variant="im")
    out.append((c, p))
    c, _ = W.spinodal(n=100, variant="qim", seed=4)
    c = dict(c, nx=100, ny=57)
    out.append((c, W.spinodal_phi(100, 57, 0.5, 0.05, 4)))
    c, p = W.static_droplet(n=31, R=7.0, variant="im", rho_ratio=3.0)
    out.append((dict(c, fsurf="mu_grad_phi", gravity=1e-6), p))
    c, _ = W.spinodal(n=129, variant="qim", seed=5)
    c = dict(c, nx=129, ny=64, pscheme="eq28_paper_g0", bc="walls_y")
    out.append((c, W.spinodal_phi(129, 64, 0.5, 0.05, 5)))
    c, p = W.layered_poiseuille(nx=16, ny=200, mu_ratio=3.0, rho_ratio=3.0, visc="step", G=1e-6)
    out.append((c, p))
    return out


def make_batch(insts):
    import torch
    from paper_1902_08933_amd import lbpf
    b = lbpf.Batch([c for c, _ in insts])
    for k, (_, phi) in enumerate(insts):
        b.init(k, torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    return b


def single(cfg, phi, steps):
    import torch
    from paper_1902_08933_amd import lbpf
    s = lbpf.Simulation(cfg)
    s.init(torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda())
    s.step(steps)
    return s


def fields(sim):
    return {f: sim.read(f).cpu().numpy() for f in ("phi", "ux", "uy", "p")}


def test_batch_bitwise_equals_single_simulations():
    insts = mixed_instances()
    b = make_batch(insts)
    b.step(21)  # two graph replays of 8 steps and five single launches
    assert b.step_count == 21
    for k, (c, p) in enumerate(insts):
        print(f"instance {k}: {c['nx']}x{c['ny']}", flush=True)
        got = fields(b.instance(k))
        ref = fields(single(c, p, 21))
        for f in got:
            np.testing.assert_array_equal(got[f], ref[f])


def test_step_each_equals_graph_replay():
    insts = mixed_instances()
    a = make_batch(insts)
    a.step(16)
    b = make_batch(insts)
    b.step_each(16)
    for k in range(len(insts)):
        fa, fb = fields(a.instance(k)), fields(b.instance(k))
        for f in fa:
            np.testing.assert_array_equal(fa[f], fb[f])


def test_batch_shapes_bit_identical():
    from paper_1902_08933_amd import lbpf
    insts = mixed_instances()[:3]
    ref = None
    for t in range(len(lbpf.tile_shapes())):
        b = make_batch(insts)
        b.set_tile(t)
        b.step(9)
        got = [fields(b.instance(k)) for k in range(len(insts))]
        if ref is None:
            ref = got
        else:
            for g, r in zip(got, ref):
                for f in g:
                    np.testing.assert_array_equal(g[f], r[f])


def test_batch_instance_matches_oracle():
    insts = mixed_instances()
    b = make_batch(insts)
    b.step(60)
    for k in (1, 4):
        c, p = insts[k]
        o = oracle.Oracle(c).init(np.asarray(p, dtype=np.float32).astype(np.float64)).step(60)
        g = b.instance(k)
        phi = g.read("phi").double().cpu().numpy()
        u = np.stack([g.read("ux").double().cpu().numpy(), g.read("uy").double().cpu().numpy()])
        ru = np.stack([o.read("ux"), o.read("uy")])
        assert np.linalg.norm(phi - o.read("phi")) / np.linalg.norm(o.read("phi")) < 1e-5
        assert np.linalg.norm(u - ru) / np.linalg.norm(ru) < 1e-5


def test_diverged_instance_is_frozen_and_others_continue():
    insts = mixed_instances()[:4]
    bad = np.array(insts[2][1], dtype=np.float32)
    bad[10, 10] = np.nan
    insts_bad = list(insts)
    insts_bad[2] = (insts[2][0], bad)
    b = make_batch(insts_bad)
    b.step(5)
    flags, diags = b.status()
    assert flags == [0, 0, 1, 0]
    assert diags[2]["nonfinite"] > 0 and diags[0]["nonfinite"] == 0
    frozen = fields(b.instance(2))
    b.step(12)
    after = fields(b.instance(2))
    for f in frozen:
        np.testing.assert_array_equal(frozen[f], after[f])
    for k in (0, 1, 3):
        got = fields(b.instance(k))
        ref = fields(single(insts[k][0], insts[k][1], 17))
        for f in got:
            np.testing.assert_array_equal(got[f], ref[f])
    # re-initializing a frozen instance brings it back
    b.init(2, insts[2][1])
    b.step(3)
    flags, _ = b.status()
    assert flags == [0, 0, 0, 0]


def test_batch_autotune_restores_state():
    insts = mixed_instances()[:3]
    a = make_batch(insts)
    a.step(10)
    best, ms = a.autotune(trial_steps=2)
    assert a.tile == best and all(t > 0 for t in ms)
    a.step(10)
    b = make_batch(insts)
    b.step(20)
    for k in range(len(insts)):
        fa, fb = fields(a.instance(k)), fields(b.instance(k))
        for f in fa:
            np.testing.assert_array_equal(fa[f], fb[f])


def test_batch_of_256_instances_runs():
    # the 256-instance workload (sides 64..512); the instances that the method cannot hold
    # stable (large density ratios) are detected and frozen, the others stay finite
    insts = W.batch_instances(256, seed=0)
    b = make_batch(insts)
    b.step(40)
    flags, diags = b.status()
    ok = [d for f, d in zip(flags, diags) if not f]
    assert len(ok) >= 100
    assert all(d["nonfinite"] == 0 for d in ok)
    print(f"256 instances: {sum(flags)} frozen after 40 steps", flush=True)


def test_every_instance_frozen_leaves_an_empty_work_list():
    # both instances go non-finite: the work list is empty, steps (graph replays and single
    # launches) do nothing, and re-initializing one brings it back alone
    insts = mixed_instances()[:2]
    bad = [(c, np.where(np.arange(p.size).reshape(p.shape) == 7, np.nan, p).astype(np.float32))
           for c, p in insts]
    b = make_batch(bad)
    b.step(3)
    flags, _ = b.status()
    assert flags == [1, 1]
    before = [fields(b.instance(k)) for k in range(2)]
    b.step(11)
    for k in range(2):
        after = fields(b.instance(k))
        for f in after:
            np.testing.assert_array_equal(before[k][f], after[f])
    b.init(0, insts[0][1])
    b.step(5)
    flags, diags = b.status()
    assert flags == [0, 1] and diags[0]["nonfinite"] == 0
    got = fields(b.instance(0))
    ref = fields(single(insts[0][0], insts[0][1], 5))
    for f in got:
        np.testing.assert_array_equal(got[f], ref[f])


def test_single_launches_then_graph_replays_keep_every_item():
    # 3 single launches leave the next counter slot at 3: the following call launches 5 singles
    # up to slot 0, then a graph replay of 8 and 6 more singles; every item must run each step
    insts = mixed_instances()[:4]
    b = make_batch(insts)
    b.step(3)
    b.step(19)
    b.step(1)
    assert b.step_count == 23
    for k, (c, p) in enumerate(insts):
        got = fields(b.instance(k))
        ref = fields(single(c, p, 23))
        for f in got:
            np.testing.assert_array_equal(got[f], ref[f])
