"""Training driver and evaluation of the learned preconditioner (all compute in the HIP library).

Training pairs come from the even-odd system Dhat(m+, m-) of the EOFA operator on seeded gauge
fields, with A = Dhat^dag Dhat: errors of early CG iterates (e_k = x* - x_k, rho_k = A e_k, made on
the device by eofa_training_pairs) and Gaussian errors e with rho = A e.  The network learns
N(rho) ~ e, an approximate inverse of A (flexible GCR applies it as z = N(Dhat^dag r)), with Adam on
the relative squared error.  Pairs are generated per gauge field and streamed: only one field's pairs
are resident at a time.

Evaluation solves H_T(m+, m-) x = b on held-out gauge fields with plain FP64 CG and with FGCR + network
and reports iterations, Dhat applications and wall time of both.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import eofa as E
from . import inputs as IN


def _gauss5(ctx, seed):
    torch = ctx.torch
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    re = torch.randn(ctx.shape5, generator=g, dtype=torch.float64)
    im = torch.randn(ctx.shape5, generator=g, dtype=torch.float64)
    return torch.complex(re, im).to(ctx.device)


def make_pairs(ctx, mp, mm, seed, n_cg=8, n_rand=4):
    """(rho, e) pairs for the current gauge field: n_cg from CG iterates, n_rand from Gaussian errors."""
    pairs = ctx.training_pairs(mp, mm, seed, n_cg) if n_cg else []
    for i in range(n_rand):
        e = _gauss5(ctx, seed * 1000 + i)
        rho = ctx.apply("SCHUR_NORMAL", e, mp, mm)
        pairs.append((rho, e))
    return pairs


def identity_init(seed, noise=0.05):
    """Parameters of a network close to the identity map: the centre tap of every layer is the unit
    matrix on the 24 live channels, plus seeded Gaussian noise of relative size `noise`; zero biases."""
    wsz, lsz = 81 * 32 * 32, 81 * 32 * 32 + 32
    p = IN.cnn_params(seed, scale=noise).astype(np.float64)
    for l in range(4):
        p[l * lsz + wsz: (l + 1) * lsz] = 0.0
        W = p[l * lsz: l * lsz + wsz].reshape(81, 32, 32)
        W[40, np.arange(24), np.arange(24)] += 1.0
    return p.astype(np.float32)


def train(ctx, fields, mp, mm, steps=1000, lr=2e-4, lr_end=2e-5, seed=0, relu=False, n_cg=0, n_rand=8,
          steps_per_field=50, init="identity", log=None):
    """Train the network of ctx in place on pairs from the gauge fields (list of (seed, links)).
    init: "identity" (near-identity linear network) or "he" (random He-normal).  Returns the loss history."""
    if init == "identity":
        ctx.set_precond(identity_init(seed), relu=relu)
    else:
        ctx.cnn_init(seed=seed, relu=relu)
    hist = []
    step = 0
    t0 = time.perf_counter()
    while step < steps:
        for fseed, U in fields:
            if step >= steps:
                break
            ctx.set_gauge(U)
            pairs = make_pairs(ctx, mp, mm, fseed * 7919 + step, n_cg, n_rand)
            for k in range(min(steps_per_field, steps - step)):
                rho, e = pairs[k % len(pairs)]
                frac = step / max(steps - 1, 1)
                rate = lr * (lr_end / lr) ** frac  # geometric decay
                hist.append(ctx.cnn_train_step(rho, e, lr=rate))
                step += 1
            if log:
                log(f"step {step}/{steps} field {fseed} loss(last {min(steps_per_field, len(hist))}) "
                    f"{np.mean(hist[-steps_per_field:]):.4f} {time.perf_counter() - t0:.1f}s")
    ctx.torch.cuda.synchronize()
    return hist


def evaluate(ctx, fields, mp, mm, tol=1e-10, nsrc=1, log=None):
    """Plain FP64 CG against FGCR + network on each (seed, links) field; returns a list of records."""
    out = []
    for fseed, U in fields:
        ctx.set_gauge(U)
        for i in range(nsrc):
            b = _gauss5(ctx, 10_000 + 100 * fseed + i)
            _, cg = ctx.solve_ht(b, mp, mm, E.params(tol=tol))
            _, fg = ctx.solve_ht(b, mp, mm, E.params(tol=tol, pc=E.PC_LEARNED))
            rec = dict(field=fseed, src=i, cg=cg, fgcr=fg,
                       iter_ratio=cg["iters"] / max(fg["iters"], 1),
                       apply_ratio=cg["op_applies"] / max(fg["op_applies"], 1),
                       time_ratio=cg["seconds"] / max(fg["seconds"], 1e-12))
            out.append(rec)
            if log:
                log(f"field {fseed} src {i}: CG {cg['iters']} it / {cg['op_applies']} Dhat / {cg['seconds']:.3f}s; "
                    f"FGCR+CNN {fg['iters']} it / {fg['op_applies']} Dhat / {fg['seconds']:.3f}s "
                    f"(fell back: {fg['fell_back']})")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--lr", type=float, default=2e-4)
    ap.add_argument("--n-cg", type=int, default=0, help="pairs per field from CG iterates")
    ap.add_argument("--n-rand", type=int, default=8, help="pairs per field from Gaussian errors")
    ap.add_argument("--relu", action="store_true")
    ap.add_argument("--save", default=None, help="write the trained parameters (float32 .npy)")
    ap.add_argument("--json", default=None, help="write the evaluation records")
    a = ap.parse_args(argv)
    cfg = IN.CONFIGS[a.config]
    dims, Ns, eps = cfg["dims"], cfg["Ns"], cfg["eps"]
    mp, mm = cfg["masses"][0], cfg["masses"][1]
    log = lambda m: print(m, flush=True)
    ctx = E.Context(dims, Ns, IN.M0, IN.optimal_omega(Ns))
    train_f = [(s, IN.gauge_links(dims, eps, s)) for s in cfg["train_seeds"]]
    hold_f = [(s, IN.gauge_links(dims, eps, s)) for s in cfg["heldout_seeds"]]
    t0 = time.perf_counter()
    hist = train(ctx, train_f, mp, mm, steps=a.steps, lr=a.lr, relu=a.relu, n_cg=a.n_cg, n_rand=a.n_rand, log=log)
    t_train = time.perf_counter() - t0
    recs = evaluate(ctx, hold_f, mp, mm, log=log)
    summary = dict(config=a.config, steps=a.steps, train_seconds=t_train, final_loss=float(np.mean(hist[-50:])),
                   iter_ratio=float(np.mean([r["iter_ratio"] for r in recs])),
                   apply_ratio=float(np.mean([r["apply_ratio"] for r in recs])),
                   time_ratio=float(np.mean([r["time_ratio"] for r in recs])))
    print(json.dumps(summary), flush=True)
    if a.save:
        np.save(a.save, ctx.cnn_params())
    if a.json:
        with open(a.json, "w") as f:
            json.dump(dict(summary=summary, records=recs, loss=hist), f)


if __name__ == "__main__":
    main()
