"""Profiling driver for the fused even-odd hop (run it under rocprofv3).

    python -m paper_1710_09621_amd.profile_hop [--dims 32 32 32 64] [--Ns 16] [--nrep 10] [--sched 1,1,4,4,8,32,0 ...]
                                               [--all] [--cg N]

Sets up the seeded lattice, autotunes the hop schedule (or takes the given ones, or with --all every schedule the
autotuner would time, one after the other),
launches the FP64 hop nrep times per schedule
(the kernel behind the bench's dslash figure) and then applies the site-local A_T^{-1}
(k_site: one streaming read and one streaming write of a half field per parity, the same
access pattern as the hop's spinor traffic) once, so that hardware byte counters can be
calibrated against a kernel of known traffic in the same process.  With --cg N it then runs the benchmark's
step once under the last schedule: the source build and even-odd preparation of the action (+1, 0.01, 0.1, 1.0)
followed by exactly N FP64 CG iterations (kernels K1..K5 of each iteration, eofa_cg_block), and prints their
launch counts and algorithmic bytes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[32, 32, 32, 64])
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--eps", type=float, default=0.7)
    ap.add_argument("--nrep", type=int, default=10)
    ap.add_argument("--prec", type=int, default=0)
    ap.add_argument("--sched", action="append", default=[],
                    help="fixed schedule (7 comma-separated ints); repeat to time several in one process")
    ap.add_argument("--all", action="store_true", help="every candidate schedule of the autotuner, in its order")
    ap.add_argument("--cg", type=int, default=0, help="then N FP64 CG iterations of the benchmark step")
    args = ap.parse_args()
    import numpy as np
    import torch
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    dims = tuple(args.dims)
    U = IN.gauge_links(dims, args.eps, 5)
    ctx = E.Context(dims, args.Ns, IN.M0, IN.optimal_omega(args.Ns))
    ctx.set_gauge(U)
    scheds = [[int(v) for v in sc.split(",")] for sc in args.sched]
    if args.all:
        scheds += ctx.schedule_candidates(prec=args.prec)
    if not scheds:
        scheds = [ctx.autotune(prec=args.prec)["sched"]]
    Vh = int(np.prod(dims)) // 2
    for sched in scheds:
        ctx.set_schedule(sched, prec=args.prec)
        r = ctx.dslash_bench(nrep=args.nrep, prec=args.prec)
        print(json.dumps(dict(dims=dims, Ns=args.Ns, prec=args.prec, schedule=sched, ms=r["ms"], gbs=r["gbs"],
                              alg_bytes=r["bytes"], site_kernel_bytes_each_way=Vh * 12 * args.Ns * 16)), flush=True)
    x = torch.randn(ctx.shape5, dtype=torch.complex128, device="cuda")
    ctx.apply("AT_INV", x, 0.01, 0.01)
    torch.cuda.synchronize()
    if args.cg:
        phi = torch.from_numpy(IN.gaussian_spinor(dims[::-1], 11)).cuda()
        ctx.kernel_timing(True, reset=True)
        rel = ctx.cg_block(+1, 0.01, 0.1, phi, args.cg)
        st = ctx.kernel_timing(False)
        print(json.dumps(dict(dims=dims, Ns=args.Ns, schedule=scheds[-1], cg_iters=args.cg, rel=rel,
                              kernels={k: dict(launches=v["launches"], bytes=v["bytes"]) for k, v in st.items()})),
              flush=True)


if __name__ == "__main__":
    main()
