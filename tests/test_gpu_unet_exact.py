"""Bitwise checks of the surrogate's convolution kernels against the FP64 oracle, layer by layer.

Inputs are small integers / 8 and weights small integers / 8, so every product is a multiple of
1/64 and every FP32 accumulation of up to 9 x 384 products (and of the 2 x 2 pool and the fused
1 x 1 head) is exact, whatever the order of summation. The oracle's FP64 convolution then gives
the same numbers exactly: the FP32 outputs must be bitwise equal to it, and the bf16 outputs
bitwise equal to its round-to-nearest-even. Shapes include the layer shapes of the 1024 x 1024
inference pass, which select the kernel variants that pass runs (each test asserts the variant).
"""
import zlib

import numpy as np
import pytest

from oracle import unet_oracle as U

pytestmark = pytest.mark.gpu


def bits(a):
    """bf16 bit patterns (int16) of float64 values that are exactly representable in bf16"""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32)
    assert np.all((u & 0xFFFF) == 0), "value not exact in bf16"
    return (u >> 16).astype(np.uint16).view(np.int16)


def from_bits(t):
    """float64 values of a tensor of bf16 bit patterns"""
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def small(rng, shape, lo, hi):
    return rng.integers(lo, hi + 1, size=shape).astype(np.float64) / 8.0


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def run_conv(rng, ks, n, h, w, cin, cout, cl=0, relu=True, pool=False, head_rc=0, first=0, net=False):
    """one convolution through lbpf_unet_conv_probe and its exact FP64 reference; with net, only
    the outputs the network's own layer writes (y and its pool, or with a head the prediction
    alone), which selects the kernels' specialized output paths"""
    import torch
    from paper_1902_08933_amd import lbpf
    wt = small(rng, (cout, ks * ks, cin), -2, 2)
    bias = small(rng, (cout,), -4, 4)
    args = {}
    if first:
        xin = small(rng, (n, h, w, first), -4, 4)
        wt[:, :, first:] = 0.0  # the first layer's weights beyond the input fields are unused
        x_full = np.zeros((n, h, w, cin))
        x_full[..., :first] = xin
        args["xin"] = dev(xin.astype(np.float32))
    else:
        x = small(rng, (n, h, w, cin - cl), -4, 4)
        args["x"] = dev(bits(x))
        x_full = x
        if cl:
            xl = small(rng, (n, h // 2, w // 2, cl), -4, 4)
            args["xl"] = dev(bits(xl))
            x_full = np.concatenate([U.up(xl), x], axis=-1)
    out = U.conv(x_full, wt, bias)  # FP64, exact
    if relu:
        out = np.maximum(out, 0.0)
    y = None if (net and head_rc) else torch.empty((n, h, w, cout), dtype=torch.int16, device="cuda")
    yf = None if net else torch.empty((n, h, w, cout), dtype=torch.float32, device="cuda")
    yp = torch.empty((n, h // 2, w // 2, cout), dtype=torch.int16, device="cuda") if pool else None
    extra = {}
    if head_rc:
        hw = small(rng, (head_rc, cout), -2, 2)
        hb = small(rng, (head_rc,), -4, 4)
        res = small(rng, (n, h, w, head_rc), -8, 8)
        pred = torch.empty((n, h, w, head_rc), dtype=torch.float32, device="cuda")
        extra = dict(hw=dev(bits(hw)), hb=dev(hb.astype(np.float32)), res=dev(res.astype(np.float32)), pred=pred)
    variant = lbpf.conv_probe(ks, relu, n, h, w, cin, cout, dev(bits(wt)), cl=cl,
                              bias=dev(bias.astype(np.float32)), y=y, yf=yf, yp=yp, **args, **extra)
    torch.cuda.synchronize()
    got, exp = {}, {}
    if yf is not None:
        got["yf"], exp["yf"] = yf.double().cpu().numpy(), out
    if y is not None:
        got["y"], exp["y"] = from_bits(y), U.bf16_round(out)
    if pool:
        got["yp"] = from_bits(yp)
        exp["yp"] = U.bf16_round(U.pool(U.bf16_round(out)))
    if head_rc:
        got["pred"] = extra["pred"].double().cpu().numpy()
        exp["pred"] = res + hb + U.bf16_round(out) @ hw.T
    return variant, got, exp


def assert_bitwise(got, exp):
    for k in exp:
        g = got[k].astype(np.float32)
        e = exp[k].astype(np.float32)
        assert np.array_equal(g.view(np.uint32), e.view(np.uint32)), \
            (k, int((g != e).sum()), float(np.abs(g - e).max()))


# (name, kwargs, expected variant (kernel: 0 tiled, 1 first layer, 2 wave-row, 3 persistent first
# layer; output channels per workgroup; weight prefetch of the tiled kernel, or 8-row work items
# of the wave-row kernel))
CASES = [
    # the first layer of the 1024^2 pass: FP32 fields in, (tap, field)-ordered K; the persistent
    # kernel when only y and its pool are written (the network's case), whole tiles, 4 fields
    ("first_1024", dict(ks=3, n=1, h=1024, w=1024, cin=16, cout=32, first=4, pool=True, net=True), (3, 32, 0)),
    ("first_loop_images", dict(ks=3, n=3, h=48, w=80, cin=16, cout=32, first=4, pool=True, net=True, relu=False),
     (3, 32, 0)),
    ("first_fp32_out", dict(ks=3, n=1, h=64, w=64, cin=16, cout=32, first=4, pool=True), (1, 32, 0)),
    ("first_cout64", dict(ks=3, n=2, h=40, w=24, cin=16, cout=64, first=3), (1, 64, 0)),
    # the 3x3 layers of the 1024^2 pass run the wave-row kernel (whole 32-channel chunks):
    # E1 (level 1, 32 -> 64, one input chunk, fused pool), E2 (64 -> 128), E3 (128 -> 256),
    # D2 ([up(E3), E2] 384 -> 128) and D1 ([up(D2), E1] 192 -> 64) with the upsampling fused,
    # D0 ([up(D1), E0] 96 -> 32) with the fused 1 x 1 head and prediction; 1024^2 D0 has four
    # work items per workgroup, so the persistent loop and its chunk pipeline across items run
    ("enc1_512", dict(ks=3, n=1, h=512, w=512, cin=32, cout=64, pool=True), (2, 64, 0)),
    ("enc2_256", dict(ks=3, n=1, h=256, w=256, cin=64, cout=128, pool=True), (2, 128, 0)),
    ("enc3_128", dict(ks=3, n=1, h=128, w=128, cin=128, cout=256), (2, 128, 1)),
    ("dec2_256", dict(ks=3, n=1, h=256, w=256, cin=384, cl=256, cout=128), (2, 128, 0)),
    ("dec1_512", dict(ks=3, n=1, h=512, w=512, cin=192, cl=128, cout=64), (2, 64, 0)),
    ("dec0_head_1024", dict(ks=3, n=1, h=1024, w=1024, cin=96, cl=64, cout=32, head_rc=4), (2, 32, 0)),
    # the same layers with only the outputs the network writes (the output paths specialized
    # at compile time: y; y and its pool; the head's prediction alone)
    ("enc1_512_net", dict(ks=3, n=1, h=512, w=512, cin=32, cout=64, pool=True, net=True), (2, 64, 0)),
    ("enc2_256_net", dict(ks=3, n=1, h=256, w=256, cin=64, cout=128, pool=True, net=True), (2, 128, 0)),
    ("enc3_128_net", dict(ks=3, n=1, h=128, w=128, cin=128, cout=256, net=True), (2, 128, 1)),
    ("dec2_256_net", dict(ks=3, n=1, h=256, w=256, cin=384, cl=256, cout=128, net=True), (2, 128, 0)),
    ("dec1_512_net", dict(ks=3, n=1, h=512, w=512, cin=192, cl=128, cout=64, net=True), (2, 64, 0)),
    ("dec0_head_1024_net", dict(ks=3, n=1, h=1024, w=1024, cin=96, cl=64, cout=32, head_rc=4, net=True),
     (2, 32, 0)),
    ("dec0_head_ragged_net", dict(ks=3, n=2, h=40, w=72, cin=96, cl=64, cout=32, head_rc=4, net=True), (2, 32, 0)),
    ("wave32_ragged_pool_net", dict(ks=3, n=3, h=24, w=72, cin=64, cout=32, pool=True, net=True), (2, 32, 0)),
    # ragged tiles (rows and columns beyond the image), several images, no activation, a head
    # with rc != 4, the pool at every channel grouping, images of one patch
    ("dec0_head_ragged", dict(ks=3, n=2, h=40, w=72, cin=96, cl=64, cout=32, head_rc=4), (2, 32, 0)),
    ("wave_head_rc3", dict(ks=3, n=1, h=20, w=70, cin=64, cl=32, cout=32, head_rc=3), (2, 32, 0)),
    ("wave32_ragged_pool", dict(ks=3, n=3, h=24, w=72, cin=64, cout=32, pool=True), (2, 32, 0)),
    ("wave64_ragged_pool", dict(ks=3, n=2, h=34, w=50, cin=96, cl=32, cout=64, pool=True, relu=False), (2, 64, 0)),
    ("wave128_ragged_pool", dict(ks=3, n=1, h=18, w=30, cin=32, cout=384, pool=True), (2, 128, 1)),
    ("wave128_half_ragged", dict(ks=3, n=2, h=26, w=40, cin=64, cl=32, cout=128, pool=True, net=True), (2, 128, 1)),
    ("wave128_full_ragged", dict(ks=3, n=8, h=60, w=72, cin=64, cout=256, pool=True), (2, 128, 0)),
    ("wave32_one_patch", dict(ks=3, n=2, h=18, w=66, cin=32, cout=32), (2, 32, 0)),
    # the tiled kernel, which takes images smaller than one patch of the wave-row kernel (with
    # the fused head) and channel counts that are not whole 32-channel chunks: COT 64
    # with the weight prefetch, COT 32 with and without it (three workgroups per CU on a grid of
    # at least 768 workgroups), and COT 16 (the 1 x 1 head of the training pass, FP32 outputs,
    # no activation)
    ("tile64_cin40", dict(ks=3, n=2, h=256, w=256, cin=40, cl=16, cout=64, pool=True), (0, 64, 1)),
    ("tile32_cin48_ragged", dict(ks=3, n=3, h=24, w=72, cin=48, cout=32, pool=True), (0, 32, 1)),
    ("tile32_head_small", dict(ks=3, n=2, h=40, w=24, cin=96, cl=64, cout=32, head_rc=4), (0, 32, 1)),
    ("tile32_tiny", dict(ks=3, n=1, h=4, w=6, cin=32, cout=32), (0, 32, 1)),
    ("tile32_cin24_large", dict(ks=3, n=1, h=512, w=512, cin=24, cout=40), (0, 32, 0)),
    ("head_1x1_cout16", dict(ks=1, n=2, h=48, w=40, cin=32, cout=16, relu=False), (0, 16, 1)),
]


@pytest.mark.parametrize("name,kw,variant", CASES, ids=[c[0] for c in CASES])
def test_conv_kernel_bitwise(name, kw, variant):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    print(f"conv probe {name}: {kw}", flush=True)
    got_variant, got, exp = run_conv(rng, **kw)
    print(f"  variant {got_variant}", flush=True)
    assert got_variant == variant
    assert_bitwise(got, exp)


@pytest.mark.parametrize("ks,n,h,w,cin,cout,chunks", [(3, 2, 64, 64, 64, 64, 64), (3, 1, 40, 24, 32, 32, 8),
                                                      (1, 2, 48, 48, 32, 16, 16), (3, 1, 128, 128, 128, 256, 64)])
def test_wgrad_kernel_bitwise(ks, n, h, w, cin, cout, chunks):
    from paper_1902_08933_amd import lbpf
    rng = np.random.default_rng(ks * 1000 + cin + cout)
    x = small(rng, (n, h, w, cin), -4, 4)
    dy = small(rng, (n, h, w, cout), -4, 4)
    wt = np.zeros((cout, ks * ks, cin))
    _, gw, gb = U.conv_backward(x, wt, dy)  # FP64, exact
    print(f"wgrad probe ks {ks} {n}x{h}x{w} {cin}->{cout}, {chunks} chunks", flush=True)
    dw, db = lbpf.wgrad_probe(ks, dev(bits(dy)), dev(bits(x)), n, h, w, cin, cout, max_chunks=chunks)
    assert_bitwise({"dw": dw.double().cpu().numpy(), "db": db.double().cpu().numpy()}, {"dw": gw, "db": gb})


def test_conv_probe_rejects_unaligned_channels():
    import torch
    from paper_1902_08933_amd import lbpf
    wt = torch.zeros((16, 9, 12), dtype=torch.int16, device="cuda")
    x = torch.zeros((1, 16, 16, 12), dtype=torch.int16, device="cuda")
    with pytest.raises(lbpf.LbpfError):
        lbpf.conv_probe(3, True, 1, 16, 16, 12, 16, wt, x=x,
                        y=torch.empty((1, 16, 16, 16), dtype=torch.int16, device="cuda"))
