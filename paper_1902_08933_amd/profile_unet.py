"""Profiling driver for the surrogate network (run it under rocprofv3 --kernel-trace --stats):
forward passes at one resolution, optionally training steps.

python -m paper_1902_08933_amd.profile_unet --h 1024 --w 1024 --reps 10
python -m paper_1902_08933_amd.profile_unet --train --batch 8 --h 256 --w 256 --reps 10
"""
import argparse
import sys

import numpy as np

from . import lbpf


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=int, default=1024)
    ap.add_argument("--w", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--train", action="store_true")
    a = ap.parse_args()
    net = lbpf.UNet(max_batch=a.batch, max_h=a.h, max_w=a.w, train=a.train, seed=1)
    g = torch.Generator().manual_seed(0)
    x = (torch.randn(a.batch, a.h, a.w, 4, generator=g) * 0.1).cuda()
    y = x * 0.9
    if a.train:
        net.train_step(x, y, 1e-4)
    else:
        out = torch.empty_like(x)
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
