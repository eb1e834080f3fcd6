"""GPU (HIP C ABI) against the FP64 oracle: operators element by element, solves by the oracle's residual."""
import numpy as np
import pytest

from gpu_common import ctx_and_oracle, rand5, relerr

pytestmark = pytest.mark.gpu

# (dims, Ns): several 256-lane tiles plus ragged tails; Ns = 4, 8, 16 (DPP path), 32
CASES = [((4, 4, 4, 4), 8), ((4, 4, 4, 8), 16), ((2, 2, 2, 6), 4), ((6, 4, 2, 4), 16), ((4, 2, 2, 4), 32)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}_Ns{c[1]}")
def setup(request):
    dims, Ns = request.param
    print(f"[gpu] case dims={dims} Ns={Ns}", flush=True)
    return ctx_and_oracle(dims, Ns)


MASSES = [(0.05, 0.05), (0.01, 0.3), (1.0, 0.1)]


@pytest.mark.parametrize("mp,mm", MASSES)
def test_dt_and_friends(setup, mp, mm):
    ctx, lat = setup
    x = rand5(lat, 3)
    assert relerr(ctx.apply("DT", x, mp, mm), lat.dt(x, mp, mm)) < 1e-12
    assert relerr(ctx.apply("DT_DAG", x, mp, mm), lat.dt(x, mp, mm, dag=True)) < 1e-12
    assert relerr(ctx.apply("HT", x, mp, mm), lat.ht(x, mp, mm)) < 1e-12
    assert relerr(ctx.apply("AT_INV", x, mp, mm), lat.at_inv(x, mp, mm)) < 1e-12


@pytest.mark.parametrize("mp,mm", MASSES)
def test_dodwf(setup, mp, mm):
    """The optimal-DWF operator D_odwf = D_w omega (1 + L) + (1 - L) and its adjoint (the oracle forms them from
    the definition; the library from A - (1/2) H omega (1 + L) with site-local tables)."""
    ctx, lat = setup
    x = rand5(lat, 7)
    assert relerr(ctx.apply("DODWF", x, mp, mm), lat.dodwf(x, mp, mm)) < 1e-12
    assert relerr(ctx.apply("DODWF_DAG", x, mp, mm), lat.dodwf(x, mp, mm, dag=True)) < 1e-12


def test_parity_hops(setup):
    """H_eo and H_oe: the hop of the odd (even) half into the even (odd) sites; the other half of out is zero
    and the input's own half is not read."""
    from oracle import oracle as O
    ctx, lat = setup
    x = rand5(lat, 8)
    odd = O.parity_mask(lat.dims)[None, ..., None, None]
    hop = lambda f: np.stack([lat.hop(f[s]) for s in range(lat.Ns)])
    assert relerr(ctx.apply("HOP_EO", x), hop(x * odd) * ~odd) < 1e-12
    assert relerr(ctx.apply("HOP_OE", x), hop(x * ~odd) * odd) < 1e-12
    assert np.all(ctx.apply("HOP_EO", x).cpu().numpy()[np.broadcast_to(odd, x.shape)] == 0)


def test_dw_and_hop(setup):
    ctx, lat = setup
    x = rand5(lat, 4)
    ref_dw = np.stack([lat.dw(x[s]) for s in range(lat.Ns)])
    ref_hop = np.stack([lat.hop(x[s]) for s in range(lat.Ns)])
    assert relerr(ctx.apply("DW", x), ref_dw) < 1e-12
    assert relerr(ctx.apply("HOP", x), ref_hop) < 1e-12


@pytest.mark.parametrize("mp,mm", MASSES[:2])
def test_schur(setup, mp, mm):
    from oracle import oracle as O
    ctx, lat = setup
    odd = O.parity_mask(lat.dims)[None, ..., None, None]
    x = rand5(lat, 5) * odd
    s = lat.schur(x, mp, mm)
    assert relerr(ctx.apply("SCHUR", x, mp, mm), s) < 1e-12
    assert relerr(ctx.apply("SCHUR_DAG", x, mp, mm), lat.schur(x, mp, mm, dag=True)) < 1e-12
    assert relerr(ctx.apply("SCHUR_NORMAL", x, mp, mm), lat.schur(s, mp, mm, dag=True)) < 1e-12


def test_solve_ht_residual(setup):
    from paper_1710_09621_amd import eofa as E
    ctx, lat = setup
    b = rand5(lat, 6)
    for mp, mm in [(0.01, 0.01), (0.02, 0.5)]:
        x, info = ctx.solve_ht(b, mp, mm, E.params(max_iter=20000))
        xn = x.cpu().numpy()
        res = np.linalg.norm(b - lat.ht(xn, mp, mm)) / np.linalg.norm(b)
        assert res <= 1e-10, (res, info)
        assert info["true_rel_resid"] <= 1e-10
        assert abs(info["true_rel_resid"] - res) < 1e-11


# Oracle solves are unpreconditioned CG on the full lattice: keep their volumes small.
SOLVE_CASES = [((4, 4, 4, 4), 8), ((2, 2, 2, 6), 4), ((2, 2, 2, 4), 16), ((2, 2, 2, 4), 32)]


@pytest.fixture(scope="module", params=SOLVE_CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}_Ns{c[1]}")
def small(request):
    dims, Ns = request.param
    print(f"[gpu] solve case dims={dims} Ns={Ns}", flush=True)
    return ctx_and_oracle(dims, Ns)


@pytest.mark.parametrize("chir,m3,m4,mo", [(-1, 0.05, 0.05, 1.0), (+1, 0.01, 0.1, 1.0), (-1, 1.0, 0.1, 1.0)])
def test_chiral_action(small, chir, m3, m4, mo):
    """Solutions agree with the oracle's to the solver tolerance: both reach a true residual of
    1e-12, so outputs agree to ~cond * 1e-12; 1e-9 relative leaves a 1000x condition margin."""
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = small
    phi = IN.gaussian_spinor(lat.shape4[:-2], 11)
    r = ctx.chiral_action(chir, m3, m4, mo, phi, E.params(tol=1e-12, max_iter=20000))
    ref, S, info = lat.chiral_action(chir, m3, m4, mo, phi, tol=1e-12)
    assert r.info[0]["true_rel_resid"] <= 1e-12
    assert relerr(r.out, ref) < 1e-9
    assert abs(r.S - S) < 1e-9 * abs(S)


def test_hinv(small):
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = small
    phi = IN.gaussian_spinor(lat.shape4[:-2], 12)
    r = ctx.hinv(phi, 0.05, 1.0, E.params(tol=1e-12, max_iter=20000))
    ref, S, info = lat.hinv(phi, 0.05, 1.0, tol=1e-12)
    assert relerr(r.out, ref) < 1e-9
    assert abs(r.S - S) < 1e-9 * abs(S)
    assert r.S > 0


# ---------------------------------------------------------------- FP32 storage and the mixed solver
FP32_TOL = 2e-6  # FP32 unit roundoff 6e-8 times the ~30-term depth of hop + ring scan


@pytest.mark.parametrize("mp,mm", MASSES[:2])
def test_fp32_operators(setup, mp, mm):
    from oracle import oracle as O
    from paper_1710_09621_amd import eofa as E
    ctx, lat = setup
    x = rand5(lat, 21)
    F = E.MIXED_FP32
    assert relerr(ctx.apply("DT", x, mp, mm, prec=F), lat.dt(x, mp, mm)) < FP32_TOL
    assert relerr(ctx.apply("DT_DAG", x, mp, mm, prec=F), lat.dt(x, mp, mm, dag=True)) < FP32_TOL
    assert relerr(ctx.apply("AT_INV", x, mp, mm, prec=F), lat.at_inv(x, mp, mm)) < FP32_TOL
    odd = O.parity_mask(lat.dims)[None, ..., None, None]
    xo = x * odd
    s = lat.schur(xo, mp, mm)
    assert relerr(ctx.apply("SCHUR", xo, mp, mm, prec=F), s) < FP32_TOL
    assert relerr(ctx.apply("SCHUR_NORMAL", xo, mp, mm, prec=F), lat.schur(s, mp, mm, dag=True)) < FP32_TOL


def test_mixed_solve_reaches_fp64_residual(setup):
    from paper_1710_09621_amd import eofa as E
    ctx, lat = setup
    b = rand5(lat, 22)
    for mp, mm in [(0.01, 0.01), (0.02, 0.5)]:
        x, info = ctx.solve_ht(b, mp, mm, E.params(tol=1e-10, prec=E.MIXED_FP32, max_iter=40000))
        xn = x.cpu().numpy()
        res = np.linalg.norm(b - lat.ht(xn, mp, mm)) / np.linalg.norm(b)
        assert res <= 1e-10, (res, info)
        assert info["reliable_updates"] >= 2
        x64, _ = ctx.solve_ht(b, mp, mm, E.params(tol=1e-10))
        assert relerr(x, x64.cpu().numpy()) < 1e-7


def test_mixed_chiral_action(small):
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = small
    phi = IN.gaussian_spinor(lat.shape4[:-2], 13)
    r = ctx.chiral_action(+1, 0.01, 0.1, 1.0, phi, E.params(tol=1e-12, prec=E.MIXED_FP32, max_iter=40000))
    ref, S, info = lat.chiral_action(+1, 0.01, 0.1, 1.0, phi, tol=1e-12)
    assert r.info[0]["true_rel_resid"] <= 1e-12
    assert relerr(r.out, ref) < 1e-9
    assert abs(r.S - S) < 1e-9 * abs(S)
