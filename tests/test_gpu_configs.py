"""The other synthetic workloads at their full sizes: the 16^3 x 32 precision comparison and the
24^3 x 48 multi-RHS batch (12 sources over 3 mass pairs = 24 systems, FP32 storage, hipGraph replay).
Every solve must reach the FP64 true residual; solutions of each workload are checked with the oracle's own
H_T on the whole lattice (one FP64 solve at 16^3 x 32, one batched FP32 solve per mass pair at 24^3 x 48), and
the reduced-precision results against FP64 GPU solves."""
import numpy as np
import pytest
import torch

from gpu_common import relerr

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _setup(cfg_id):
    from oracle import oracle as O
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    cfg = IN.CONFIGS[cfg_id]
    U = IN.gauge_links(cfg["dims"], cfg["eps"], cfg["seed"])
    om = IN.optimal_omega(cfg["Ns"])
    ctx = E.Context(cfg["dims"], cfg["Ns"], IN.M0, om)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    lat = O.Lattice(cfg["dims"], U, m0=IN.M0, omega=om, tbc=-1)
    return cfg, ctx, lat


def test_config2_precisions():
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    print("[gpu] config 2: 16^3x32 Ns=16", flush=True)
    cfg, ctx, lat = _setup(2)
    m_lo, m_hi = cfg["masses"]
    phis = [torch.from_numpy(IN.gaussian_spinor(cfg["dims"][::-1], 2000 + j)) for j in range(cfg["nsrc"])]
    for j, phi in enumerate(phis):
        r64 = ctx.hinv(phi, m_lo, m_hi, E.params(tol=1e-10))
        for prec in (E.MIXED_FP32, E.MIXED_FP16):
            r = ctx.hinv(phi, m_lo, m_hi, E.params(tol=1e-10, prec=prec))
            assert all(i["true_rel_resid"] <= 1e-10 for i in r.info)
            err = relerr(r.out, r64.out.cpu().numpy())
            print(f"  source {j} prec {prec}: |out - out_fp64| / |out_fp64| = {err:.1e}, "
                  f"iters {[i['iters'] for i in r.info]} vs {[i['iters'] for i in r64.info]}")
            assert err < 1e-8 and abs(r.S - r64.S) <= 1e-9 * abs(r64.S)
    # one FP64 5D solve verified by the oracle's operator on the whole lattice
    rng = np.random.default_rng(2100)
    b = rng.standard_normal(lat.shape5) + 1j * rng.standard_normal(lat.shape5)
    x, info = ctx.solve_ht(torch.from_numpy(b), m_lo, m_hi, E.params(tol=1e-10))
    res = lat.ht(x.cpu().numpy(), m_lo, m_hi) - b
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(b)


def test_config3_batched_graph_fp32():
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    print("[gpu] config 3: 24^3x48 Ns=16, 24 systems", flush=True)
    cfg, ctx, lat = _setup(3)
    ctx.autotune(prec=E.MIXED_FP32)
    pairs, phis = [], []
    for k, pr in enumerate(cfg["pairs"]):
        for j in range(cfg["nsrc"]):
            pairs.append(pr)
            phis.append(torch.from_numpy(IN.gaussian_spinor(cfg["dims"][::-1], 3000 + 10 * k + j)))
    res = ctx.hinv_batch(pairs, phis, E.params(tol=1e-10, prec=E.MIXED_FP32, use_graph=1))
    assert len(res) == 12
    for r in res:
        assert all(i["true_rel_resid"] <= 1e-10 for i in r.info)
    print(f"  graph stats {ctx.graph_stats()}; iterations {[r.info[0]['iters'] for r in res]}")
    for k in range(3):  # the first source of each mass pair against a single FP64 solve
        j = k * cfg["nsrc"]
        r64 = ctx.hinv(phis[j], *pairs[j], E.params(tol=1e-10))
        assert relerr(res[j].out, r64.out.cpu().numpy()) < 1e-8
        assert abs(res[j].S - r64.S) <= 1e-9 * abs(r64.S)
    del res, phis
    # the same batched FP32 hipGraph path on 5D systems: one H_T per mass pair (the + system of each pair, the
    # larger mass second), every solution checked with the oracle's own H_T on the whole lattice
    systems = [(lo, hi) for lo, hi in cfg["pairs"]]
    rng = np.random.default_rng(3100)
    bs = [rng.standard_normal(lat.shape5) + 1j * rng.standard_normal(lat.shape5) for _ in systems]
    out = ctx.solve_ht_batch(systems, [torch.from_numpy(b) for b in bs],
                             E.params(tol=1e-10, prec=E.MIXED_FP32, use_graph=1))
    for (x, info), b, (mp, mm) in zip(out, bs, systems):
        res = lat.ht(x.cpu().numpy(), mp, mm) - b
        rel = np.linalg.norm(res) / np.linalg.norm(b)
        print(f"  H_T({mp}, {mm}): iters {info['iters']}, GPU residual {info['true_rel_resid']:.2e}, "
              f"oracle residual {rel:.2e}")
        assert info["true_rel_resid"] <= 1e-10 and rel <= 2e-10
