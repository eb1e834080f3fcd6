"""FP16-column storage of the Krylov vectors (EOFA_MIXED_FP16): FP32 arithmetic, FP64 reliable
updates, so every solve must still reach the FP64 true residual; checked with the oracle's operator."""
import numpy as np
import pytest
import torch

from gpu_common import ctx_and_oracle, rand5, relerr

pytestmark = pytest.mark.gpu

CASES = [((4, 4, 4, 4), 8), ((4, 4, 4, 8), 16), ((4, 2, 2, 4), 32), ((6, 4, 2, 4), 16)]


@pytest.mark.parametrize("dims,Ns", CASES, ids=lambda c: str(c))
@pytest.mark.parametrize("mp,mm", [(0.01, 0.1), (1.0, 0.1)])
def test_fp16_solve_reaches_fp64_residual(dims, Ns, mp, mm):
    from paper_1710_09621_amd import eofa as E
    print(f"[gpu] fp16 solve dims={dims} Ns={Ns} masses=({mp}, {mm})", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    b = rand5(lat, 31)
    x16, i16 = ctx.solve_ht(torch.as_tensor(b), mp, mm, E.params(tol=1e-10, prec=E.MIXED_FP16))
    x64, i64 = ctx.solve_ht(torch.as_tensor(b), mp, mm, E.params(tol=1e-10))
    print(f"  fp16 {i16}\n  fp64 {i64}")
    assert i16["true_rel_resid"] <= 1e-10
    r = lat.ht(x16.cpu().numpy(), mp, mm) - b
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)
    assert relerr(x16, x64.cpu().numpy()) < 1e-8


def test_fp16_batch_matches_fp64():
    from paper_1710_09621_amd import eofa as E
    dims, Ns = (4, 4, 4, 8), 16
    print(f"[gpu] fp16 batch dims={dims} Ns={Ns}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    rng = np.random.default_rng(32)
    phis = [torch.as_tensor(rng.standard_normal(lat.shape4) + 1j * rng.standard_normal(lat.shape4)) for _ in range(3)]
    acts = [(-1, 0.01, 0.01, 0.1), (1, 0.01, 0.1, 1.0), (-1, 1.0, 0.1, 0.1)]
    r64 = ctx.chiral_action_batch(acts, phis, E.params(tol=1e-11))
    for graph in (0, 1):
        r16 = ctx.chiral_action_batch(acts, phis, E.params(tol=1e-11, prec=E.MIXED_FP16, use_graph=graph))
        for a, b in zip(r64, r16):
            assert b.info[0]["true_rel_resid"] <= 1e-11
            assert relerr(b.out, a.out.cpu().numpy()) < 1e-8
            assert abs(a.S - b.S) <= 1e-9 * abs(a.S)
