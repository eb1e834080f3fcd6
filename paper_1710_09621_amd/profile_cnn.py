"""Profiling driver for the learned preconditioner's convolution kernels (run it under rocprofv3).

    python paper_1710_09621_amd/profile_cnn.py [--dims 16 16 16 32] [--Ns 16] [--nrep 5]

Sets up the seeded 16^3 x 32, Ns = 16 lattice, installs seeded network parameters, then runs the
network forward nrep times (four k_conv_fwd launches each) and nrep training steps (forward, weight
gradient, backward-data convolutions and Adam), timing both with HIP events on the library's stream.
Prints the per-call times and the convolution flop rate against the dense BF16 matrix-core peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# per site and s-slice: 81 taps x 2 x (24*32 + 32*32 + 32*32 + 32*24) multiply-adds
FLOP_PER_ROW = 81 * 2 * (24 * 32 + 32 * 32 + 32 * 32 + 32 * 24)
BF16_PEAK_TFLOPS = 2500.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--nrep", type=int, default=5)
    args = ap.parse_args()
    import numpy as np
    import torch
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    dims = tuple(args.dims)
    ctx = E.Context(dims, args.Ns, IN.M0, IN.optimal_omega(args.Ns))
    ctx.set_gauge(IN.gauge_links(dims, args.eps, 4))
    ctx.set_precond(IN.cnn_params(1))
    g = torch.Generator(device="cpu").manual_seed(3)
    x = torch.complex(torch.randn(ctx.shape5, generator=g, dtype=torch.float64),
                      torch.randn(ctx.shape5, generator=g, dtype=torch.float64)).to("cuda")
    e = torch.complex(torch.randn(ctx.shape5, generator=g, dtype=torch.float64),
                      torch.randn(ctx.shape5, generator=g, dtype=torch.float64)).to("cuda")
    ctx.cnn_apply(x)
    ctx.cnn_train_step(x, e, lr=1e-5)
    st = ctx.stream
    res = {}
    for name, fn in (("apply", lambda: ctx.cnn_apply(x)), ("train_step", lambda: ctx.cnn_train_step(x, e, lr=1e-5))):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(st)
        for _ in range(args.nrep):
            fn()
        t1.record(st)
        torch.cuda.synchronize()
        res[name + "_ms"] = t0.elapsed_time(t1) / args.nrep
    rows = int(np.prod(dims)) // 2 * args.Ns
    tf = rows * FLOP_PER_ROW / 1e12
    res.update(dims=dims, Ns=args.Ns, rows=rows, forward_tflop=tf,
               apply_tflops=tf / (res["apply_ms"] * 1e-3), peak_tflops=BF16_PEAK_TFLOPS)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
