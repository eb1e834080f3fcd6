"""HMC of one-flavour QCD with the exact one-flavor action and mass preconditioning (Sec. I; Sec. III).

    python -m paper_1710_09621_amd.hmc [--config 2] [--scheme new] [--ntraj 2] [--steps 480 12 6] [--beta 6.2]
    python -m paper_1710_09621_amd.hmc --config 2 --therm 30 --compare --ntraj 4   # the three splittings of Sec. III

Every trajectory follows the outline of Sec. I:
  (2) momenta P^a ~ N(0, 1) and (3) pseudofermion noise eta of weight exp(-eta^dag eta), drawn on the host from
      seeded generators (the draws are inputs of the library);
  (4) every pseudofermion field phi = A^{-1/2} P_c eta from the heat-bath of its chiral action
      (eofa_chiral_heatbath);
  (5) the molecular dynamics with the Omelyan integrator nested over three time scales and (6) the Metropolis
      test, both in eofa_md_trajectory.
The levels follow Sec. III: the gauge field at k0, the last (heaviest) factor of the splitting at k1, the other
factors at k2, with (k0, k1, k2) = (480, 12, 6).  Prints one JSON line per trajectory and a summary per splitting
with the CG iterations, the time and the force magnitudes (|F| averaged over the links; per action the largest
and the mean over its evaluations in a trajectory, and the gauge force), the quantities Sec. III compares.
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


def levels(acts):
    """(level, chir, m3, m4, mo) per chiral action of a splitting: the last factor at level 1, the others at 2."""
    return [(1 if i == len(acts) - 1 else 2,) + tuple(a) for i, a in enumerate(acts)]


def trajectory(ctx, U, acts, rng, beta, tau, steps, p, chrono=True, force_tol=0.0, hb_err=1e-10, metropolis=True):
    """One HMC trajectory in place on U (device links): momenta and noise from rng, the heat-bath of every
    action, the molecular dynamics and the Metropolis test.  Returns the trajectory's record."""
    import numpy as np
    import torch
    Lx, Ly, Lz, Lt = ctx.dims
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = torch.from_numpy(rng.standard_normal((4, Lt, Lz, Ly, Lx, 8))).cuda()
    phis, hb = [], []
    for (lev, chir, m3, m4, mo) in acts:
        eta = (rng.standard_normal((Lt, Lz, Ly, Lx, 4, 3)) + 1j * rng.standard_normal((Lt, Lz, Ly, Lx, 4, 3)))
        eta *= np.sqrt(0.5)  # weight exp(-eta^dag eta)
        phi, info = ctx.chiral_heatbath(chir, m3, m4, mo, eta, rel_err=hb_err, p=p)
        phis.append(phi)
        hb.append(info)
    torch.cuda.synchronize()
    t_hb = time.perf_counter() - t0
    u = float(rng.random())
    md = ctx.md_trajectory(U, P, [a + (phis[i],) for i, a in enumerate(acts)], beta, tau, steps,
                           metropolis_u=u if metropolis else -1.0,
                           p=p, chrono=chrono, force_tol=force_tol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plaq = 1.0 - ctx.gauge_action(U, 1.0) / (6 * Lx * Ly * Lz * Lt)
    n = min(len(acts), 8)
    return dict(dH=md["dH"], accepted=md["accepted"], u=u, plaquette=plaq, seconds=round(t, 3),
                heatbath_s=round(t_hb, 3), md_s=round(md["seconds"], 3), cg_iters=md["cg_iters"],
                force_evals=md["force_evals"][:len(steps)], link_updates=md["link_updates"],
                hb_poles=[h["npoles"] for h in hb], H0=md["H0"], Sg0=md["Sg0"], Sf0=md["Sf0"],
                force_max=[round(v, 6) for v in md["force_max"][:n]],
                force_mean=[round(v, 6) for v in md["force_mean"][:n]], gauge_force0=round(md["gauge_force0"], 6))


def summarize(lines, dims, Ns, scheme, acts, args):
    import numpy as np
    summary = dict(lattice="x".join(map(str, dims)), Ns=Ns, scheme=scheme, actions=[list(a) for a in acts],
                   beta=args.beta, steps=args.steps, prec=args.prec, ntraj=len(lines), chrono=not args.no_chrono,
                   force_tol=args.force_tol, hb_err=args.hb_err,
                   accepted=sum(1 for x in lines if x["accepted"] == 1),
                   mean_s=round(sum(x["seconds"] for x in lines) / len(lines), 3),
                   mean_cg=round(sum(x["cg_iters"] for x in lines) / len(lines), 1),
                   force_max=[round(float(v), 5) for v in np.mean([x["force_max"] for x in lines], axis=0)],
                   force_mean=[round(float(v), 5) for v in np.mean([x["force_mean"] for x in lines], axis=0)],
                   gauge_force0=round(float(np.mean([x["gauge_force0"] for x in lines])), 5))
    eq = lines[args.burn:]
    if len(eq) >= 2:
        # every proposal counts in <exp(-dH)>, which is 1 in equilibrium for a reversible, area-preserving
        # integrator; jackknife error over single trajectories
        w = np.exp(-np.array([x["dH"] for x in eq]))
        n = len(w)
        jk = (w.sum() - w) / (n - 1)
        err = float(np.sqrt((n - 1) / n * np.sum((jk - jk.mean()) ** 2)))
        summary.update(burn=args.burn, exp_mdH=float(w.mean()), exp_mdH_err=err,
                       acceptance=sum(1 for x in eq if x["accepted"] == 1) / n,
                       plaquette=float(np.mean([x["plaquette"] for x in eq])),
                       mean_abs_dH=float(np.mean([abs(x["dH"]) for x in eq])))
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2, help="synthetic start field and lattice (inputs.CONFIGS)")
    ap.add_argument("--dims", type=int, nargs=4, default=None)
    ap.add_argument("--Ns", type=int, default=None)
    ap.add_argument("--scheme", choices=("none", "old", "new"), default="new")
    ap.add_argument("--compare", action="store_true",
                    help="after --therm trajectories of --scheme, run --ntraj trajectories of each splitting (new, "
                         "old, none), every one starting from the same thermalised field")
    ap.add_argument("--schemes", default="new,old,none", help="the splittings --compare runs, in order")
    ap.add_argument("--therm", type=int, default=0, help="trajectories before the measured ones (reported as such)")
    ap.add_argument("--therm-nomet", action="store_true",
                    help="keep the end point of every thermalisation trajectory (no Metropolis test), for rough starts")
    ap.add_argument("--therm-m", type=float, default=None, help="light mass of the thermalisation (default --m)")
    ap.add_argument("--therm-mh", type=float, default=None, help="heavy mass of the thermalisation (default --mh)")
    ap.add_argument("--m", type=float, default=0.01)
    ap.add_argument("--mh", type=float, default=0.1)
    ap.add_argument("--M", type=float, default=1.0)
    ap.add_argument("--beta", type=float, default=6.2)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--steps", type=int, nargs=3, default=[480, 12, 6])
    ap.add_argument("--ntraj", type=int, default=2)
    ap.add_argument("--prec", choices=("fp64", "fp16"), default="fp16")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=None, help="also write the lines to this file")
    ap.add_argument("--force-tol", type=float, default=1e-8,
                    help="residual target of the interior force solves (0: the actions' 1e-10)")
    ap.add_argument("--hb-err", type=float, default=1e-10,
                    help="relative error of the rational approximation of x^(-1/2) in the heat-bath")
    ap.add_argument("--no-chrono", action="store_true",
                    help="start every force solve from zero instead of the action's previous solution")
    ap.add_argument("--burn", type=int, default=0,
                    help="trajectories left out of the equilibrium averages (<exp(-dH)>, acceptance, plaquette)")
    args = ap.parse_args()

    import numpy as np
    import torch
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    from paper_1710_09621_amd import mpseq

    cfg = IN.CONFIGS[args.config]
    dims = tuple(args.dims or cfg["dims"])
    Ns = args.Ns or cfg["Ns"]
    Lx, Ly, Lz, Lt = dims
    U = torch.from_numpy(IN.gauge_links(dims, cfg["eps"], cfg["seed"]).reshape(Lt, Lz, Ly, Lx, 4, 3, 3)).cuda()
    ctx = E.Context(dims, Ns, IN.M0, IN.optimal_omega(Ns))
    ctx.set_gauge(U)
    prec = {"fp64": E.FP64, "fp16": E.MIXED_FP16}[args.prec]
    p = E.params(tol=1e-10, prec=prec, max_iter=50000)

    def splitting(kind, m=args.m, mh=args.mh):
        return levels(mpseq.actions(kind, m, [] if kind == "none" else [mh], args.M))

    tm = args.m if args.therm_m is None else args.therm_m
    tmh = args.mh if args.therm_mh is None else args.therm_mh

    rng = np.random.Generator(np.random.PCG64(args.seed))
    out = []

    def emit(x):
        out.append(x)
        print(json.dumps(x), flush=True)

    for traj in range(args.therm):
        emit(dict(phase="therm", scheme=args.scheme, traj=traj, masses=[tm, tmh, args.M],
                  **trajectory(ctx, U, splitting(args.scheme, tm, tmh), rng, args.beta, args.tau, args.steps, p,
                               chrono=not args.no_chrono, force_tol=args.force_tol, hb_err=args.hb_err,
                               metropolis=not args.therm_nomet)))
    start = U.clone()
    for scheme in (tuple(args.schemes.split(",")) if args.compare else (args.scheme,)):
        U.copy_(start)
        ctx.set_gauge(U)
        acts = splitting(scheme)
        lines = []
        for traj in range(args.ntraj):
            line = dict(traj=traj, scheme=scheme, **trajectory(ctx, U, acts, rng, args.beta, args.tau, args.steps, p,
                                                               chrono=not args.no_chrono, force_tol=args.force_tol,
                                                               hb_err=args.hb_err))
            lines.append(line)
            emit(line)
        emit(dict(summary=summarize(lines, dims, Ns, scheme, acts, args)))
    if args.out:
        with open(args.out, "w") as f:
            for x in out:
                f.write(json.dumps(x) + "\n")


if __name__ == "__main__":
    main()
