"""Profiling driver for the surrogate network (run it under rocprofv3 --kernel-trace --stats):
forward passes at one resolution, optionally training steps.

python -m paper_1902_08933_amd.profile_unet --h 1024 --w 1024 --warmup 100 --reps 10
python -m paper_1902_08933_amd.profile_unet --train --batch 8 --h 256 --w 256 --reps 10
"""
import argparse
import sys

import numpy as np

from . import lbpf


def forward_flop(n, h, w, base=32):
    """FLOPs (2 per multiply-add) of one forward pass of the network at n x h x w: per layer,
    pixels at its level x Cout x KS^2 x Cin (layer table of the library's network)."""
    c = [base << l for l in range(4)]
    layers = [(0, 16, c[0], 3), (1, c[0], c[1], 3), (2, c[1], c[2], 3), (3, c[2], c[3], 3),
              (2, c[3] + c[2], c[2], 3), (1, c[2] + c[1], c[1], 3), (0, c[1] + c[0], c[0], 3),
              (0, c[0], 16, 1)]
    return sum(2 * n * (h >> lev) * (w >> lev) * co * ks * ks * ci for lev, ci, co, ks in layers)


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=int, default=1024)
    ap.add_argument("--w", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed passes first (the clocks settle over about 100 forward passes)")
    ap.add_argument("--train", action="store_true")
    ap.add_argument("--flop-only", action="store_true",
                    help="print the multiply-add FLOPs of one forward pass and exit (no GPU)")
    a = ap.parse_args()
    if a.flop_only:
        print(forward_flop(a.batch, a.h, a.w))
        return 0
    net = lbpf.UNet(max_batch=a.batch, max_h=a.h, max_w=a.w, train=a.train, seed=1)
    g = torch.Generator().manual_seed(0)
    x = (torch.randn(a.batch, a.h, a.w, 4, generator=g) * 0.1).cuda()
    y = x * 0.9
    out = None if a.train else torch.empty_like(x)
    for _ in range(max(1, a.warmup)):
        if a.train:
            net.train_step(x, y, 1e-4)
        else:
            net.forward(x, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.reps):
        if a.train:
            net.train_step(x, y, 1e-4)
        else:
            net.forward(x, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.reps
    print(f"{'train step' if a.train else 'forward'} {a.batch}x{a.h}x{a.w}: {ms:.3f} ms", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
