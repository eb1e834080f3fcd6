"""The t-walk hop schedules (workgroups walking t with the backward t term carried, modes 3, 5 and 6) against the
default schedule and the oracle: every operator bit-for-bit equal to the default schedule's in FP64 and
FP32 for every t-walk schedule the autotuner may pick, the FP64 D_T against the oracle, and a CG solve
under a t-walk schedule checked by the oracle's residual."""
import numpy as np
import pytest
import torch

from gpu_common import ctx_and_oracle, rand5, relerr

pytestmark = pytest.mark.gpu

# lattices on which t-walk schedules exist (a t-slab holds a whole number of 256-lane segments);
# several chunks of 16 slabs, Ns = 8, 16 (DPP lane exchange), 32 (ds_bpermute); (32, 4, 4, 16) at Ns = 16 has
# the benchmark's x-line length (16 sites per parity, one line per segment)
CASES = [((8, 8, 8, 32), 16), ((8, 8, 8, 32), 8), ((16, 8, 4, 16), 32), ((32, 4, 4, 16), 16)]
OPS = ["DW", "HOP", "DT", "DT_DAG", "HT", "AT_INV", "SCHUR", "SCHUR_DAG", "SCHUR_NORMAL"]


def tw_schedules(dims, Ns):
    """The t-walk candidates of the autotuner: [3, 5 or 6, xcd, ty, tz, tt, nyb, KB of reserved LDS]."""
    Lxh, Ly, Lz, Lt = dims[0] // 2, dims[1], dims[2], dims[3]
    if (Lxh * Ly * Ns) % 256:
        return []
    nyb = Lxh * Ly * Ns // 256
    out = []
    for ty in (1, 2, 4, 8, 16):
        for tz in (1, 2, 4, 8, 16):
            if not 8 <= ty * tz <= 64 or nyb % ty or Lz % tz:
                continue
            for tt in sorted({16, Lt}):
                if Lt % tt:
                    continue
                for pad in (0, 48):
                    # 5: x neighbours from LDS, segments of whole x-lines; 6: the same with the spin-split lanes
                    # (Ns = 16); both hold a CU's LDS, so they take no reserve
                    for mode in (3, 5, 6):
                        if mode >= 5 and ((256 // Ns) % Lxh or pad):
                            continue
                        if mode == 6 and Ns != 16:
                            continue
                        out.append([mode, 1, ty, tz, tt, nyb, pad])
    return out


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}_Ns{c[1]}")
def setup(request):
    dims, Ns = request.param
    print(f"[gpu] t-walk case dims={dims} Ns={Ns}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    return ctx, lat, dims, Ns


def test_schedules_exist(setup):
    _, _, dims, Ns = setup
    assert len(tw_schedules(dims, Ns)) >= 4


def test_candidate_list(setup):
    """The library's list of autotuner candidates starts with the two linear orders, holds exactly the t-walk
    schedules enumerated above for FP64 / FP32 and none for FP16 storage, and every entry installs."""
    from paper_1710_09621_amd import eofa as E
    ctx, _, dims, Ns = setup
    for p in (E.FP64, E.MIXED_FP32, E.MIXED_FP16):
        c = ctx.schedule_candidates(prec=p)
        assert [s[:2] for s in c[:2]] == [[0, 0], [0, 1]]
        tw = sorted(s for s in c if s[0] >= 3)
        assert tw == (sorted(tw_schedules(dims, Ns)) if p != E.MIXED_FP16 else []), p
        assert len({tuple(s) for s in c}) == len(c)
        for s in c:
            ctx.set_schedule(s, prec=p)
        ctx.set_schedule(c[0], prec=p)
    with pytest.raises(E.EofaError):
        ctx.schedule_candidates(prec=7)


@pytest.mark.parametrize("prec", ["FP64", "MIXED_FP32"])
def test_operators_equal_default_schedule(setup, prec):
    from paper_1710_09621_amd import eofa as E
    ctx, lat, dims, Ns = setup
    p = getattr(E, prec)
    x = torch.from_numpy(rand5(lat, 11)).cuda()
    base = {op: ctx.apply(op, x, 0.05, 0.3, prec=p) for op in OPS}
    default = [0, 0, 1, 1, 1, Ns * dims[0] * dims[1] // 512, 0]
    try:
        for sc in tw_schedules(dims, Ns):
            ctx.set_schedule(sc, prec=p)
            for op in OPS:
                y = ctx.apply(op, x, 0.05, 0.3, prec=p)
                assert torch.equal(y, base[op]), (sc, op)
    finally:
        ctx.set_schedule(default, prec=p)


def test_fp64_dt_against_oracle(setup):
    from paper_1710_09621_amd import eofa as E
    ctx, lat, dims, Ns = setup
    default = [0, 0, 1, 1, 1, Ns * dims[0] * dims[1] // 512, 0]
    x = rand5(lat, 12)
    try:
        ctx.set_schedule(tw_schedules(dims, Ns)[0], prec=E.FP64)
        assert relerr(ctx.apply("DT", x, 0.01, 0.1), lat.dt(x, 0.01, 0.1)) < 1e-12
        assert relerr(ctx.apply("HT", x, 0.01, 0.1), lat.ht(x, 0.01, 0.1)) < 1e-12
    finally:
        ctx.set_schedule(default, prec=E.FP64)


def test_solve_under_twalk(setup):
    """The CG reductions (per-workgroup partial norms over a whole t-walk, so summed in another order than
    under the default schedule) and the solve: oracle residual within the tolerance, iterations as under
    the default schedule up to the rounding of the reductions."""
    from paper_1710_09621_amd import eofa as E
    ctx, lat, dims, Ns = setup
    default = [0, 0, 1, 1, 1, Ns * dims[0] * dims[1] // 512, 0]
    b = rand5(lat, 13)
    x0, info0 = ctx.solve_ht(b, 0.02, 0.3, E.params(max_iter=20000))
    try:
        ctx.set_schedule(tw_schedules(dims, Ns)[-1], prec=E.FP64)
        x1, info1 = ctx.solve_ht(b, 0.02, 0.3, E.params(max_iter=20000))
    finally:
        ctx.set_schedule(default, prec=E.FP64)
    res = np.linalg.norm(b - lat.ht(x1.cpu().numpy(), 0.02, 0.3)) / np.linalg.norm(b)
    assert res <= 1e-10, (res, info1)
    assert abs(info1["iters"] - info0["iters"]) <= 2, (info0, info1)
    assert relerr(x1, x0.cpu().numpy()) < 1e-8
