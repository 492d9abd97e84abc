"""Surrogate kernels against the FP64 CPU oracle: the MFMA operand layout bit-exactly on integer
data, the network's forward pass and its parameter gradients (BF16 storage, FP32 accumulation,
so within BF16 tolerances), training on a fixed batch, and the solver/surrogate hand-over."""
import numpy as np
import pytest

from oracle import unet_oracle as U

pytestmark = pytest.mark.gpu


def bf16_bits(a):
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


@pytest.mark.parametrize("k", [16, 32])
def test_mfma_operand_layout_exact(k):
    import torch
    from paper_1902_08933_amd import lbpf
    rng = np.random.default_rng(0)
    for trial in range(4):
        A = rng.integers(-8, 9, size=(16, k)).astype(np.float64)
        B = rng.integers(-8, 9, size=(k, 16)).astype(np.float64)
        tA = torch.from_numpy(bf16_bits(A).copy()).cuda()
        tB = torch.from_numpy(bf16_bits(B).copy()).cuda()
        D = torch.empty((16, 16), dtype=torch.float32, device="cuda")
        lbpf.mfma_probe(tA, tB, D, k=k)
        np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), A @ B)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_params(net, rng, head_scale=0.2):
    """He-normal weights for every layer including the head, small random biases"""
    L = net.layers()
    p = np.zeros(net.nparam)
    for i, l in enumerate(L):
        nw = l["cout"] * l["ks"] ** 2 * l["cin"]
        fan = l["ks"] ** 2 * (4 if i == 0 else l["cin"])
        w = rng.normal(size=nw) * np.sqrt(2.0 / fan) * (head_scale if i == 7 else 1.0)
        if i == 0:
            w = w.reshape(l["cout"], 9, l["cin"])
            w[:, :, 4:] = 0.0
            w = w.ravel()
        p[l["woff"]:l["woff"] + nw] = w
        p[l["boff"]:l["boff"] + l["cout"]] = rng.normal(size=l["cout"]) * 0.05
    return U.bf16_round(p)


def test_forward_and_gradients_match_oracle():
    import torch
    from paper_1902_08933_amd import lbpf
    rng = np.random.default_rng(1)
    n, h, w = 2, 16, 24
    net = lbpf.UNet(max_batch=n, max_h=h, max_w=w, train=True, wgrad_chunks=8, seed=3)
    p = random_params(net, rng)
    net.set_params(torch.from_numpy(p.astype(np.float32)))
    x = U.bf16_round(rng.normal(size=(n, h, w, 4)))
    tgt = x + rng.normal(size=x.shape) * 0.1
    tx = torch.from_numpy(x.astype(np.float32)).cuda()
    tt = torch.from_numpy(tgt.astype(np.float32)).cuda()
    pred = net.forward(tx).double().cpu().numpy()
    ref, _ = U.forward(p, x, base=32)
    e = rel(pred - x, ref - x)
    print(f"forward change rel L2 {e:.3e}", flush=True)
    assert e < 2e-2
    loss, g = net.loss_grad(tx, tt)
    lref, gref = U.loss_grad(p, x, tgt, base=32)
    g = g.double().cpu().numpy()
    print(f"loss {loss:.6e} vs {lref:.6e}", flush=True)
    assert abs(loss - lref) / lref < 2e-2
    cos = float(g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref)))
    print(f"gradient rel L2 {rel(g, gref):.3e} cosine {cos:.6f}", flush=True)
    assert cos > 0.999
    assert rel(g, gref) < 4e-2
    for i, l in enumerate(net.layers()):
        sl = slice(l["woff"], l["boff"] + l["cout"])
        ei = rel(g[sl], gref[sl])
        print(f"  layer {i} grad rel L2 {ei:.3e}", flush=True)
        assert ei < 6e-2


@pytest.mark.parametrize("n,h,w", [(1, 40, 24), (3, 16, 72)])
def test_inference_forward_matches_oracle(n, h, w):
    # inference networks fuse the decoder upsampling into the convolutions and write the
    # prediction from the head; sizes with partial 16 x 16 tiles at every level
    import torch
    from paper_1902_08933_amd import lbpf
    rng = np.random.default_rng(11 + n)
    net = lbpf.UNet(max_batch=n, max_h=h, max_w=w, train=False, seed=3)
    p = random_params(net, rng)
    net.set_params(torch.from_numpy(p.astype(np.float32)))
    x = U.bf16_round(rng.normal(size=(n, h, w, 4)))
    pred = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).double().cpu().numpy()
    ref, _ = U.forward(p, x, base=32)
    e = rel(pred - x, ref - x)
    print(f"inference forward {n}x{h}x{w}: change rel L2 {e:.3e}", flush=True)
    assert e < 2e-2


def test_training_fits_a_fixed_batch():
    import torch
    from paper_1902_08933_amd import lbpf
    rng = np.random.default_rng(2)
    n, h, w = 4, 32, 32
    net = lbpf.UNet(max_batch=n, max_h=h, max_w=w, train=True, seed=5)
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    x = np.stack([np.sin(2 * np.pi * (xx + k) / w)[..., None] * np.ones((1, 1, 4)) for k in range(n)])
    x = x + 0.1 * rng.normal(size=x.shape)
    tgt = np.roll(x, 1, axis=2) * 0.9  # a fixed local map the network can learn
    tx = torch.from_numpy(x.astype(np.float32)).cuda()
    tt = torch.from_numpy(tgt.astype(np.float32)).cuda()
    l0 = net.train_step(tx, tt, 1e-3)
    for _ in range(400):
        l1 = net.train_step(tx, tt, 1e-3)
    print(f"loss {l0:.4e} -> {l1:.4e}", flush=True)
    assert l1 < 0.2 * l0


def test_fields_handover_roundtrip():
    import torch
    from paper_1902_08933_amd import lbpf, workloads
    cfg, phi = workloads.spinodal(n=64, seed=1, amplitude=0.05)
    sim = lbpf.Simulation(cfg).init(torch.from_numpy(phi.astype(np.float32)).cuda())
    sim.step(200)
    shift, scale = [0.5, 0.0, 0.0, 0.0], [0.5, 1e-3, 1e-3, 1e-3]
    a = lbpf.fields_to_nhwc(sim, shift, scale)
    ref = {f: sim.read(f).double().cpu().numpy() for f in ("phi", "ux", "uy", "p")}
    an = a.double().cpu().numpy()
    np.testing.assert_allclose(an[..., 0] * 0.5 + 0.5, ref["phi"], rtol=0, atol=1e-6)
    np.testing.assert_allclose(an[..., 1] * 1e-3, ref["ux"], rtol=1e-5, atol=1e-12)
    # a new state from the same fields is the equilibrium with those fields: phi is reproduced
    # exactly up to FP32 rounding, u and p up to the non-equilibrium parts of the old state
    lbpf.init_from_nhwc(sim, a, shift, scale, step=250)
    assert sim.step_count == 250
    phi2 = sim.read("phi").double().cpu().numpy()
    assert np.abs(phi2 - ref["phi"]).max() < 1e-6
