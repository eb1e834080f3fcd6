"""Benchmark of the EOFA solve hot path on one MI355X.

Workload: the 32^3 x 64, Ns = 16 lattice (links exp(i 0.7 theta_a t^a), seeded), m0 = 1.3, the R5-symmetric
optimal weights for [0.05, 6.2], and the new mass-preconditioned sequence of Eq.(new_MP) with
(m, m_h, M) = (0.01, 0.1, 1.0): chiral actions (m,m)/(m,m_h) [-], (m,m_h)/(M,m_h) [+], (M,m_h)/(M,M) [-].

One step = the source build and even-odd preparation of the middle action (its 5D system H_T(m, m_h) needs the
most CG iterations of the three) followed by --niter FP64 CG iterations on its Schur normal equations, with no
host synchronisation inside the step.  Every kernel of every iteration is timed with HIP events on the
library's stream.  value = algorithmic GB/s of the FP64 dslash (K1, the fused even-odd hop with its A_T^{-1}
epilogue) over the timed steps.

Once per invocation, outside the timed steps, the whole sequence is solved to a true residual of 1e-10 on one
Gaussian source in plain FP64 CG and in the tuned solver (the three systems in one multi-RHS launch sequence,
FP16-column Krylov storage with FP32 arithmetic and FP64 reliable updates, autotuned schedules, hipGraph blocks
of 16 iterations); their times and iteration counts go into "tts".  Then one HMC trajectory of the same
splitting on the 16^3 x 32 workload (heat-bath, three-scale Omelyan molecular dynamics, Metropolis) goes into
"hmc".  Inputs are generated on the host and moved to HBM before anything is timed.  Prints one JSON line.
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
HOP_FLOP_PER_SITE = 1320 + 250  # Wilson hop per site and slice + the A_T^{-1} epilogue


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(U, dims, Ns, omega, budget_s=12.0):
    """The FP64 oracle's Wilson hop on s-slices of the same lattice, timed on the host cores.
    Bytes per output 5D site are counted exactly as for the GPU hop (in + out + links/Ns)."""
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
        return round(float(entry[t["by_schedule_fields"].index("bytes_per_launch")]))
    except (OSError, KeyError, ValueError):
        return None


def learned_leg(E, IN, ctx, Ns, omega, eps, action, phi_d, plain, max_iter):
    """The learned preconditioner on the step's action: the network is trained on the GPU (forward, backward and
    Adam kernels of the library) on residual->error pairs from CG iterates of 4 seeded 8^4 fields (the network
    is translation invariant), then used as the right preconditioner of flexible GCR with CG as its fallback,
    FP64, to the same true residual; its time is compared with the plain FP64 CG solve of the same action."""
    from paper_1710_09621_amd import learned as LRN
    t0 = time.perf_counter()
    small = (8, 8, 8, 8)
    ctx_t = E.Context(small, Ns, IN.M0, omega, device="cuda:0")
    fields = [(s, IN.gauge_links(small, eps, s)) for s in range(40, 44)]
    hist = LRN.train(ctx_t, fields, action[1], action[2], steps=400, lr=2e-4, lr_end=2e-5, n_cg=8, n_rand=0)
    ctx.set_precond(ctx_t.cnn_params())
    del ctx_t
    t1 = time.perf_counter()
    r = ctx.chiral_action(*action, phi_d, E.params(tol=1e-10, max_iter=max_iter, pc=E.PC_LEARNED))
    t2 = time.perf_counter()
    i = r.info[0]
    log(f"  [learned] action {action}: iters={i['iters']} fell_back={i['fell_back']} resid={i['true_rel_resid']:.2e} "
        f"{t2 - t1:.2f}s against plain {plain.info[0]['seconds']:.2f}s (training {t1 - t0:.1f}s)")
    return {"action": list(action), "s": round(t2 - t1, 3), "iters": i["iters"], "fell_back": i["fell_back"],
            "true_rel_resid": i["true_rel_resid"], "plain_fp64_s": round(plain.info[0]["seconds"], 3),
            "plain_iters": plain.info[0]["iters"], "speedup_vs_plain": round(plain.info[0]["seconds"] / (t2 - t1), 3),
            "max_rel_dS": abs(r.S - plain.S) / abs(plain.S), "training_s": round(t1 - t0, 1),
            "final_loss": float(sum(hist[-50:]) / 50),
            "form": "flexible GCR with the 4-layer BF16 convolutional network, FP64, CG fallback; trained on "
                    "CG-iterate residual->error pairs of 4 seeded 8^4 fields (400 Adam steps)"}


def hmc_leg(E, IN, max_iter):
    """One HMC trajectory of one-flavour QCD with the new-MP splitting (Sec. I; Sec. III) on the 16^3 x 32,
    Ns = 16 workload: heat-bath of the three chiral actions, the molecular dynamics with the Omelyan integrator
    on the time scales (k0, k1, k2) = (480, 12, 6) of Sec. III, and the Metropolis test; FP16-storage solves to
    1e-10 for the actions in H and 1e-8 for the interior forces, with chronological starts.  The start field is the
    synthetic one (not thermalised)."""
    import numpy as np
    import torch
    from paper_1710_09621_amd import hmc as HM
    from paper_1710_09621_amd import mpseq
    cfg = IN.CONFIGS[2]
    dims, Ns = tuple(cfg["dims"]), cfg["Ns"]
    Lx, Ly, Lz, Lt = dims
    U = torch.from_numpy(IN.gauge_links(dims, cfg["eps"], cfg["seed"]).reshape(Lt, Lz, Ly, Lx, 4, 3, 3)).cuda()
    ctx = E.Context(dims, Ns, IN.M0, IN.optimal_omega(Ns))
    ctx.set_gauge(U)
    p = E.params(tol=1e-10, prec=E.MIXED_FP16, max_iter=max_iter)
    acts = HM.levels(mpseq.actions("new", 0.01, [0.1], 1.0))
    rec = HM.trajectory(ctx, U, acts, np.random.Generator(np.random.PCG64(1)), 6.2, 1.0, [480, 12, 6], p,
                        force_tol=1e-8)
    log(f"  [hmc] trajectory {rec['seconds']:.2f}s (heat-bath {rec['heatbath_s']:.2f}s, MD {rec['md_s']:.2f}s), "
        f"dH={rec['dH']:.3f}, {rec['cg_iters']} CG iterations")
    del ctx
    torch.cuda.empty_cache()
    return dict(lattice="x".join(map(str, dims)), Ns=Ns, beta=6.2, steps=[480, 12, 6],
                actions=[list(a) for a in acts], seconds=rec["seconds"], heatbath_s=rec["heatbath_s"],
                md_s=rec["md_s"], cg_iters=rec["cg_iters"], force_evals=rec["force_evals"],
                link_updates=rec["link_updates"], dH=round(rec["dH"], 6), accepted=rec["accepted"],
                force_max=rec["force_max"], gauge_force0=rec["gauge_force0"],
                form="heat-bath + Omelyan MD on 3 time scales + Metropolis, FP16-storage solves (actions in H to 1e-10, "
                     "interior forces to 1e-8), chronological starts")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--niter", type=int, default=16, help="FP64 CG iterations per step")
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--no-tts", action="store_true", help="skip the once-per-run time-to-solution comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner leg of the time to solution")
    ap.add_argument("--no-hmc", action="store_true", help="skip the HMC trajectory leg")
    ap.add_argument("--max-iter", type=int, default=50000)
    ap.add_argument("--tune-cache", type=str, default=None)
    ap.add_argument("--tuned-prec", choices=("fp16", "fp32"), default="fp16",
                    help="Krylov storage of the tuned solver (FP32 arithmetic and FP64 reliable updates either way)")
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "hop_traffic.json"),
                    help="JSON with measured HBM bytes per hop launch (from rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the solve path has no multi-GPU form); "
                                   "run it with --gpus 1"}))
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
    phi = IN.gaussian_spinor(dims[::-1], seed * 1000)
    log(f"inputs ready in {time.time() - t0:.1f}s: dims={dims} Ns={Ns}")

    dev = torch.device("cuda:0")
    ctx = E.Context(dims, Ns, IN.M0, omega, device="cuda:0")
    ctx.set_gauge(torch.from_numpy(U).to(dev))
    phi_d = torch.from_numpy(phi).to(dev)
    if len(masses) == 3:   # new MP, Eq.(new_MP)
        m, mh, M = masses
        actions = [(-1, m, m, mh), (+1, m, mh, M), (-1, M, mh, M)]
        wl = f"EOFA new-MP sequence (m, m_h, M) = ({m}, {mh}, {M})"
    else:                  # no MP, Eq.(noMP)
        m, M = masses
        actions = [(-1, m, m, M), (+1, m, M, M)]
        wl = f"EOFA (m, m)/(M, M) = ({m}, {M}) without MP"
    # the step's system: the action whose H_T needs the most iterations (the middle one of the new MP)
    step_action = actions[1]
    tuned_prec = {"fp16": E.MIXED_FP16, "fp32": E.MIXED_FP32}[args.tuned_prec]

    # hop-kernel schedules for this lattice (in-house autotuner), outside the timed region
    tune = {}
    for prec, nm in ((E.FP64, "fp64"), (tuned_prec, args.tuned_prec)):
        ta = time.time()
        tune[nm] = ctx.autotune(prec=prec, cache=args.tune_cache)
        log(f"autotune {nm}: {tune[nm]} ({time.time() - ta:.1f}s)")

    def step():
        return ctx.cg_block(step_action[0], step_action[1], step_action[2], phi_d, args.niter)

    for w in range(args.warmup):
        ta = time.time()
        step()
        log(f"warmup step {w}: {time.time() - ta:.3f}s")
    ctx.kernel_timing(enable=True, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rel = None
    for k in range(args.steps):
        rel = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    kt = ctx.kernel_timing(enable=False)
    log(f"timed {args.steps} steps of {args.niter} CG iterations in {el:.3f}s; |r|/|r0| after a step {rel:.3e}")
    for nm, v in kt.items():
        log(f"  {nm:8s} {v['launches']:5d} launches, {v['ms'] / max(v['launches'], 1):.4f} ms each, "
            f"{v['bytes'] / max(v['ms'], 1e-12) / 1e6:.1f} GB/s")
    k1 = kt["hop"]
    hop_gbs = k1["bytes"] / (k1["ms"] * 1e-3) / 1e9
    per_launch_ms = k1["ms"] / k1["launches"]
    it_ms = sum(v["ms"] for v in kt.values()) / k1["launches"]
    it_bytes = sum(v["bytes"] for v in kt.values()) / k1["launches"]
    Vh = int(np.prod(dims)) // 2
    alg_bytes = Vh * (2 * 12 * Ns * 16 + 8 * 9 * 16)

    tts = None
    if not args.no_tts:
        P64 = E.params(tol=1e-10, max_iter=args.max_iter)
        PT = E.params(tol=1e-10, max_iter=args.max_iter, prec=tuned_prec, use_graph=1)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        plain = []
        for a in actions:
            r = ctx.chiral_action(*a, phi_d, P64)
            log(f"  [fp64] action {a}: iters={r.info[0]['iters']} resid={r.info[0]['true_rel_resid']:.2e} "
                f"S={r.S:.10e} ({r.info[0]['seconds']:.2f}s)")
            plain.append(r)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        g0 = ctx.graph_stats()
        tuned = ctx.chiral_action_batch(actions, [phi_d] * len(actions), PT)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        g1 = ctx.graph_stats()
        for a, r in zip(actions, tuned):
            log(f"  [tuned] action {a}: iters={r.info[0]['iters']} updates={r.info[0]['reliable_updates']} "
                f"resid={r.info[0]['true_rel_resid']:.2e} S={r.S:.10e}")
        resid = [r.info[0]["true_rel_resid"] for r in plain + tuned]
        dS = max(abs(a.S - b.S) / abs(a.S) for a, b in zip(plain, tuned))
        tts = {"plain_fp64_s": round(tb - ta, 3), "plain_iters": [r.info[0]["iters"] for r in plain],
               "tuned_s": round(tc - tb, 3), "tuned_iters": [r.info[0]["iters"] for r in tuned],
               "tuned": f"multi-RHS batch (the {len(actions)} systems in one launch sequence), "
                        f"{args.tuned_prec.upper()}-storage reliable-update CG, autotuned hop schedule, hipGraph "
                        f"blocks of 16 iterations ({g1['replays'] - g0['replays']} replays)",
               "speedup": round((tb - ta) / (tc - tb), 3), "max_true_rel_resid": max(resid), "max_rel_dS": dS,
               "sources": 1}
        log(f"time to solution: plain {tb - ta:.2f}s, tuned {tc - tb:.2f}s ({tts['speedup']:.2f}x)")
        if not args.no_learned:
            tts["learned"] = learned_leg(E, IN, ctx, Ns, omega, eps, step_action, phi_d, plain[1], args.max_iter)

    hmc = None
    if not args.no_hmc:
        hmc = hmc_leg(E, IN, args.max_iter)

    sched64 = tune["fp64"]["sched"]
    traffic = measured_traffic(args.traffic, dims, Ns, sched64)
    kern = {3: "k_hop_tw<16, false, HM_SITE, false, double, false> (u = A_T^{-1} H_eo p; t-walk schedule)",
            5: "k_hop_tw<16, false, HM_SITE, false, double, true> (u = A_T^{-1} H_eo p; t-walk schedule, x "
               "neighbours from LDS)",
            6: "k_hop_tws<16, false, HM_SITE, false, double> (u = A_T^{-1} H_eo p; t-walk schedule, x neighbours "
               "from LDS, two lanes per site and slice)"}.get(sched64[0],
                                                             "k_hop<16, false, HM_SITE, false, double> (u = A_T^{-1} H_eo p)")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(U, dims, Ns, omega)

    out = {
        "metric": "DWF dslash HBM GB/s; EOFA CG time-to-1e-10 residual, tuned vs plain FP64",
        "value": round(hop_gbs, 2),
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
        "config": {"workload": f"{wl}; one step = source build + even-odd preparation of the action "
                               f"{step_action} (5D system H_T({step_action[1]}, {step_action[2]})) + {args.niter} "
                               f"FP64 CG iterations on its Schur normal equations",
                   "lattice": "x".join(map(str, dims)), "Ns": Ns, "eps": eps, "seed": seed, "m0": IN.M0,
                   "cg_iterations_per_step": args.niter, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(hop_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hop_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kern, "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(per_launch_ms, 5),
                     "launches": k1["launches"],
                     "flop_per_launch": HOP_FLOP_PER_SITE * Vh * Ns,
                     "fp64_tflops": round(HOP_FLOP_PER_SITE * Vh * Ns / (per_launch_ms * 1e-3) / 1e12, 3)},
        "cg_iteration": {"ms": round(it_ms, 4), "alg_bytes": it_bytes, "gbs": round(it_bytes / it_ms / 1e6, 2),
                         "frac": round(it_bytes / it_ms / 1e6 / HBM_PEAK_GBS, 4),
                         "kernels": {nm: {"ms": round(v["ms"] / max(v["launches"], 1), 4),
                                          "gbs": round(v["bytes"] / max(v["ms"], 1e-12) / 1e6, 1)}
                                     for nm, v in kt.items()}},
        "tts": tts,
        "hmc": hmc,
        "schedules": {k: v["sched"] for k, v in tune.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
