"""Benchmark of the EOFA solve hot path on one MI355X.

One step = the new mass-preconditioned EOFA sequence of Eq.(new_MP) on the 32^3 x 64, Ns = 16
lattice (links exp(i 0.7 theta_a t^a), seeded): for (m, m_h, M) = (0.01, 0.1, 1.0) the three
chiral actions (m,m)/(m,m_h) [-], (m,m_h)/(M,m_h) [+], (M,m_h)/(M,M) [-] applied to --nsrc
Gaussian sources, every 5D solve to a true residual of 1e-10 in FP64.  Inputs are generated
on the host and moved to HBM before the timed region.

Prints one JSON line: value = FP64 dslash (fused even-odd hop) throughput in algorithmic GB/s,
measured with HIP events around every hop launch of the timed steps; roofline, CPU oracle
baseline and the time to solution of the step ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HOP_FLOP_PER_SITE = 1320 + 250


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(U, dims, Ns, omega, budget_s=12.0):
    """The FP64 oracle's Wilson hop on s-slices of the same lattice, timed on the host cores.
    Bytes per output 5D site are counted exactly as for the GPU hop (in + out + links/Ns)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1710_09621_amd import inputs as IN
    O.build()
    lat = O.Lattice(dims, U, m0=IN.M0, omega=omega)
    psi = IN.gaussian_spinor(lat.shape4[:-2], 99)
    V = lat.V
    per_site = 2 * 12 * 16 + 8 * 9 * 16 / Ns
    t0 = time.perf_counter()
    n = 0
    while True:
        lat.hop(psi)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 512:
            break
    gbs = per_site * V * n / el / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"oracle FP64 Wilson hop on the full 4D lattice {dims}, one s-slice per application, "
                      f"{n} applications in {el:.1f} s; bytes per 5D output site as for the GPU hop ({per_site:.0f} B)"}


def measured_traffic(path, dims, Ns, sched):
    """HBM bytes per launch of the dominant kernel under hop schedule sched, from the committed rocprofv3
    counter summary, or None when it has no entry for this lattice and schedule or the kernel sources
    changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        h = hashlib.sha1()
        for p in t["source_files"]:
            with open(os.path.join(ROOT, p), "rb") as f:
                h.update(f.read())
        lat = "x".join(str(d) for d in dims)
        if h.hexdigest() != t["source_sha1"] or t["lattice"] != lat or t["Ns"] != Ns:
            log("counter summary is stale (kernel sources or lattice changed): traffic = null")
            return None
        entry = t["by_schedule"].get(",".join(str(v) for v in sched))
        if entry is None:
            log(f"no counter summary for schedule {sched}: traffic = null")
            return None
        return round(float(entry["bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsrc", type=int, default=1, help="Gaussian sources per step")
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=50000)
    ap.add_argument("--tune-cache", type=str, default=None)
    ap.add_argument("--tuned-prec", choices=("fp16", "fp32"), default="fp16",
                    help="Krylov storage of the tuned solver (FP32 arithmetic and FP64 reliable updates either way)")
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "hop_traffic.json"),
                    help="JSON with measured HBM bytes per hop launch (from rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN

    cfg = IN.CONFIGS[args.config]
    dims, Ns, eps, seed = cfg["dims"], cfg["Ns"], cfg["eps"], cfg["seed"]
    masses = cfg.get("masses") or cfg["pairs"][0]
    t0 = time.time()
    U = IN.gauge_links(dims, eps, seed)
    omega = IN.optimal_omega(Ns)
    phis = [IN.gaussian_spinor(dims[::-1], seed * 1000 + j) for j in range(args.nsrc)]
    log(f"inputs ready in {time.time() - t0:.1f}s: dims={dims} Ns={Ns}")

    dev = torch.device("cuda:0")
    ctx = E.Context(dims, Ns, IN.M0, omega, device="cuda:0")
    ctx.set_gauge(torch.from_numpy(U).to(dev))
    phis_d = [torch.from_numpy(p).to(dev) for p in phis]
    if len(masses) == 3:   # new MP, Eq.(new_MP)
        m, mh, M = masses
        actions = [(-1, m, m, mh), (+1, m, mh, M), (-1, M, mh, M)]
        wl = f"EOFA new-MP solve sequence (m, m_h, M) = ({m}, {mh}, {M}), 3 chiral actions"
    else:                  # no MP, Eq.(noMP)
        m, M = masses
        actions = [(-1, m, m, M), (+1, m, M, M)]
        wl = f"EOFA (m, m)/(M, M) = ({m}, {M}) without MP, 2 chiral actions"
    P64 = E.params(tol=1e-10, max_iter=args.max_iter)
    tuned_prec = {"fp16": E.MIXED_FP16, "fp32": E.MIXED_FP32}[args.tuned_prec]
    PT = E.params(tol=1e-10, max_iter=args.max_iter, prec=tuned_prec)

    # hop-kernel schedules for this lattice (in-house autotuner), outside the timed region
    tune = {}
    for prec, nm in ((E.FP64, "fp64"), (tuned_prec, args.tuned_prec)):
        tune[nm] = ctx.autotune(prec=prec, cache=args.tune_cache)
        log(f"autotune {nm}: {tune[nm]}")

    def run(P, tag):
        res = []
        for phi in phis_d:
            for a in actions:
                ta = time.perf_counter()
                r = ctx.chiral_action(*a, phi, P)
                log(f"  [{tag}] action {a}: {time.perf_counter() - ta:.2f}s iters={r.info[0]['iters']} "
                    f"resid={r.info[0]['true_rel_resid']:.2e} S={r.S:.10e}")
                res.append(r)
        return res

    def step():
        """One pass of the hot path: the sequence in plain FP64 CG, then in the tuned solver."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.hop_timing(True)
        plain = run(P64, "fp64")
        torch.cuda.synchronize()
        ctx.hop_timing(False)
        t1 = time.perf_counter()
        acts = [a for _ in phis_d for a in actions]
        srcs = [phi for phi in phis_d for _ in actions]
        tuned = ctx.chiral_action_batch(acts, srcs, PT)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for a, r in zip(acts, tuned):
            log(f"  [tuned] action {a}: iters={r.info[0]['iters']} updates={r.info[0]['reliable_updates']} "
                f"resid={r.info[0]['true_rel_resid']:.2e} S={r.S:.10e}")
        return plain, tuned, t1 - t0, t2 - t1

    for w in range(args.warmup):
        t1 = time.time()
        step()
        log(f"warmup step {w} {time.time() - t1:.2f}s")
    torch.cuda.synchronize()
    ctx.hop_timing_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain, tuned, tp, tt = [], [], 0.0, 0.0
    for k in range(args.steps):
        a, b, x, y = step()
        plain += a
        tuned += b
        tp += x
        tt += y
        log(f"step {k} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ht = ctx.hop_timing(False)
    hop_gbs = ht["bytes"] / (ht["ms"] * 1e-3) / 1e9 if ht["ms"] > 0 else None
    per_launch_ms = ht["ms"] / max(ht["launches"], 1)
    iters = [r.info[0]["iters"] for r in plain]
    iters_t = [r.info[0]["iters"] for r in tuned]
    resid = [r.info[0]["true_rel_resid"] for r in plain + tuned]
    dS = max(abs(a.S - b.S) / abs(a.S) for a, b in zip(plain, tuned))
    log(f"timed {args.steps} steps in {el:.2f}s (plain {tp:.2f}s, tuned {tt:.2f}s); hop {ht['launches']} launches "
        f"avg {per_launch_ms:.4f} ms -> {hop_gbs:.1f} GB/s; iters {iters} / {iters_t}; max resid {max(resid):.2e}; "
        f"max |dS|/S {dS:.1e}")

    sched64 = tune["fp64"]["sched"]
    traffic = measured_traffic(args.traffic, dims, Ns, sched64)
    kern = {3: "k_hop_tw<16, false, HM_SITE, false, double, false> (u = A_T^{-1} H_eo p; t-walk schedule)",
            5: "k_hop_tw<16, false, HM_SITE, false, double, true> (u = A_T^{-1} H_eo p; t-walk schedule, x "
               "neighbours from LDS)"}.get(sched64[0], "k_hop<16, false, HM_SITE, false, double> (u = A_T^{-1} H_eo p)")

    Vh = int(np.prod(dims)) // 2
    alg_bytes = Vh * (2 * 12 * Ns * 16 + 8 * 9 * 16)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(U, dims, Ns, omega)

    out = {
        "metric": "DWF dslash HBM GB/s; EOFA CG time-to-1e-10 residual, tuned vs plain FP64",
        "value": round(hop_gbs, 2) if hop_gbs else None,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl} x {args.nsrc} Gaussian source(s), every 5D solve to a true residual of 1e-10, "
                               f"once in plain FP64 CG and once in the tuned solver",
                   "lattice": "x".join(map(str, dims)), "Ns": Ns, "eps": eps, "seed": seed, "m0": IN.M0,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(hop_gbs, 2) if hop_gbs else None, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hop_gbs / HBM_PEAK_GBS, 4) if hop_gbs else None,
                     "traffic": traffic,
                     "kernel": kern,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(per_launch_ms, 5),
                     # 1320 flop per site and slice for the Wilson hop + 250 for the A_T^{-1} epilogue
                     "flop_per_launch": HOP_FLOP_PER_SITE * Vh * Ns,
                     "fp64_tflops": round(HOP_FLOP_PER_SITE * Vh * Ns / (per_launch_ms * 1e-3) / 1e12, 3)
                     if hop_gbs else None},
        "tts": {"plain_fp64_s_per_step": round(tp / args.steps, 3), "plain_iters": iters,
                "tuned_s_per_step": round(tt / args.steps, 3), "tuned_iters": iters_t,
                "tuned": f"multi-RHS batch (all systems of the step in one launch sequence), {args.tuned_prec.upper()}-storage "
                         "reliable-update CG, autotuned hop schedule",
                "speedup": round(tp / tt, 3), "max_true_rel_resid": max(resid), "max_rel_dS": dS,
                "schedules": {k: v["sched"] for k, v in tune.items()}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
