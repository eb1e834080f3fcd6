"""Profiling driver for the EOFA fermion force (run it under rocprofv3).

    python -m paper_1710_09621_amd.profile_force [--config 5] [--nrep 2]

Sets up the seeded lattice of the workload, then computes the force of the new-MP middle action
(+, m, m_h; M) nrep times with the FP16-storage solver; the force kernel runs twice per call (one launch
per parity of the link's site).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--nrep", type=int, default=2)
    args = ap.parse_args()
    import torch
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    cfg = IN.CONFIGS[args.config]
    dims, Ns = cfg["dims"], cfg["Ns"]
    U = IN.gauge_links(dims, cfg["eps"], cfg["seed"])
    ctx = E.Context(dims, Ns, IN.M0, IN.optimal_omega(Ns))
    ctx.set_gauge(torch.from_numpy(U).cuda())
    ctx.autotune(prec=E.MIXED_FP16)
    phi = torch.from_numpy(IN.gaussian_spinor(dims[::-1], cfg["seed"] * 1000)).cuda()
    m, mh, M = 0.01, 0.1, 1.0
    for r in range(args.nrep):
        t = time.perf_counter()
        F, S, info = ctx.chiral_force(+1, m, mh, M, phi, E.params(tol=1e-10, prec=E.MIXED_FP16))
        torch.cuda.synchronize()
        print(json.dumps(dict(rep=r, s=round(time.perf_counter() - t, 3), iters=info["iters"], S=S,
                              max_abs_force=float(F.abs().max()))), flush=True)


if __name__ == "__main__":
    main()
