"""hipGraph replay of CG iteration blocks: the same kernels with the same arguments as the eager
loop, so every result must be bit-identical to the eager solve, over many replays with eager work
(residual replacement, host checks) between them."""
import numpy as np
import pytest
import torch

from gpu_common import ctx_and_oracle, rand5

pytestmark = pytest.mark.gpu

CASES = [((4, 4, 4, 4), 8), ((4, 4, 4, 8), 16)]


@pytest.mark.parametrize("dims,Ns", CASES, ids=lambda c: str(c))
@pytest.mark.parametrize("prec", ["FP64", "MIXED_FP32"])
def test_graph_solve_is_bit_identical(dims, Ns, prec):
    from paper_1710_09621_amd import eofa as E
    print(f"[gpu] graph solve dims={dims} Ns={Ns} prec={prec}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    pr = getattr(E, prec)
    b = torch.as_tensor(rand5(lat, 21))
    x0, i0 = ctx.solve_ht(b, 0.01, 0.1, E.params(tol=1e-10, prec=pr))
    g0 = ctx.graph_stats()
    for rep in range(2):  # second pass replays the cached graphs
        x1, i1 = ctx.solve_ht(b, 0.01, 0.1, E.params(tol=1e-10, prec=pr, use_graph=1))
        assert torch.equal(x0, x1), rep
        assert i1["iters"] == i0["iters"] and i1["true_rel_resid"] == i0["true_rel_resid"]
    g1 = ctx.graph_stats()
    print(f"  iters {i0['iters']}, graph stats {g0} -> {g1}")
    assert g1["replays"] - g0["replays"] >= 2 * (i0["iters"] // 16 - 2)
    assert g1["cached"] >= 1


def test_graph_batch_is_bit_identical():
    from paper_1710_09621_amd import eofa as E
    dims, Ns = (4, 4, 4, 4), 8
    print(f"[gpu] graph batch dims={dims} Ns={Ns}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    rng = np.random.default_rng(22)
    phis = [torch.as_tensor(rng.standard_normal(lat.shape4) + 1j * rng.standard_normal(lat.shape4)) for _ in range(3)]
    acts = [(-1, 0.01, 0.01, 0.1), (1, 0.01, 0.1, 1.0), (-1, 1.0, 0.1, 0.1)]
    for pr in (E.FP64, E.MIXED_FP32):
        r0 = ctx.chiral_action_batch(acts, phis, E.params(tol=1e-10, prec=pr))
        r1 = ctx.chiral_action_batch(acts, phis, E.params(tol=1e-10, prec=pr, use_graph=1))
        for a, b in zip(r0, r1):
            assert torch.equal(a.out, b.out) and a.S == b.S
    assert ctx.graph_stats()["replays"] > 0


@pytest.mark.parametrize("prec", ["FP64", "MIXED_FP32", "MIXED_FP16"])
@pytest.mark.parametrize("batch", [False, True])
def test_device_convergence_matches_every_iteration_check(prec, batch):
    """Iterations after the device has flagged convergence are skipped on the device and the iteration
    count is the device's: blocks of 16 iterations between host checks (eager and as graph replays) give
    bitwise the solution and the iteration count of a host check after every iteration."""
    from paper_1710_09621_amd import eofa as E
    dims, Ns = (4, 4, 4, 8), 16
    print(f"[gpu] device-side convergence prec={prec} batch={batch}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    pr = getattr(E, prec)
    bs = [torch.as_tensor(rand5(lat, 60 + j)) for j in range(3)]
    systems = [(0.01, 0.1), (0.1, 1.0), (1.0, 0.1)]

    def run(**kw):
        P = E.params(tol=1e-10, prec=pr, **kw)
        if batch:
            return ctx.solve_ht_batch(systems, bs, P)
        return [ctx.solve_ht(b, *m, P) for b, m in zip(bs, systems)]

    ref = run(check_every=1)
    for kw in (dict(check_every=16), dict(check_every=16, use_graph=1), dict(check_every=5, use_graph=1)):
        got = run(**kw)
        for (x0, i0), (x1, i1) in zip(ref, got):
            assert i1["iters"] == i0["iters"], (kw, i0, i1)
            assert torch.equal(x0, x1), kw
    for (x, i), b, m in zip(ref, bs, systems):
        assert i["true_rel_resid"] <= 1e-10
        r = lat.ht(x.cpu().numpy(), *m) - b.numpy()
        assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b.numpy())
