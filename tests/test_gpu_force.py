"""The EOFA fermion force through the C ABI against the oracle's force (oracle/force.py, itself pinned by
finite differences of the oracle's action): every component of every link, both chiralities, a lattice
whose t extent puts links across the antiperiodic boundary, FP64 and FP16-storage solves."""
import numpy as np
import pytest

from gpu_common import ctx_and_oracle

pytestmark = pytest.mark.gpu

CASES = [((4, 4, 4, 4), 8), ((4, 2, 2, 6), 16)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}_Ns{c[1]}")
def setup(request):
    dims, Ns = request.param
    print(f"[gpu] force case dims={dims} Ns={Ns}", flush=True)
    return ctx_and_oracle(dims, Ns)


@pytest.mark.parametrize("chir,m3,m4,mo", [(-1, 0.05, 0.05, 0.3), (+1, 0.05, 0.3, 0.6), (-1, 1.0, 0.1, 1.0)])
def test_force_fp64(setup, chir, m3, m4, mo):
    from oracle import force as OF
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = setup
    phi = IN.gaussian_spinor(lat.shape4[:-2], 31)
    F, S, info = ctx.chiral_force(chir, m3, m4, mo, phi, E.params(tol=1e-12, max_iter=20000))
    ref = OF.force(lat, chir, m3, m4, mo, phi, tol=1e-12)
    F = F.cpu().numpy()
    assert info["true_rel_resid"] <= 1e-12
    assert np.abs(F - ref).max() < 1e-9 * np.abs(ref).max()
    r = ctx.chiral_action(chir, m3, m4, mo, phi, E.params(tol=1e-12, max_iter=20000))
    assert abs(r.S - S) < 1e-12 * abs(S)


def test_force_fp16_storage(setup):
    """The force of the mixed-precision solve (true residual 1e-10) agrees to the solve's accuracy."""
    from oracle import force as OF
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = setup
    phi = IN.gaussian_spinor(lat.shape4[:-2], 32)
    F, S, info = ctx.chiral_force(+1, 0.02, 0.2, 1.0, phi, E.params(tol=1e-10, prec=E.MIXED_FP16))
    ref = OF.force(lat, +1, 0.02, 0.2, 1.0, phi, tol=1e-12)
    assert info["true_rel_resid"] <= 1e-10
    assert np.abs(F.cpu().numpy() - ref).max() < 1e-7 * np.abs(ref).max()


def test_force_rejects_null(setup):
    import ctypes as C
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    ctx, lat = setup
    phi = ctx._c128(IN.gaussian_spinor(lat.shape4[:-2], 33), ctx.shape4)
    p = E.params()
    st = ctx.lib.eofa_chiral_force(ctx.h, -1, 0.1, 0.1, 0.5, phi.data_ptr(), None, None, C.byref(p), None)
    assert st == E.EINVAL


@pytest.mark.parametrize("chir,m3,m4,mo", [(+1, 0.3, 0.6, 1.0), (-1, 0.1, 0.1, 0.5)])
def test_force_larger_lattice(chir, m3, m4, mo):
    """8x8x2x16 at Ns = 8 (whole 256-lane workgroups per (z, t) line, 32 workgroups per parity): every component
    against the oracle."""
    from oracle import force as OF
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    dims, Ns = (8, 8, 2, 16), 8
    print(f"[gpu] force case dims={dims} Ns={Ns} action={(chir, m3, m4, mo)}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns)
    phi = IN.gaussian_spinor(lat.shape4[:-2], 34)
    F, S, info = ctx.chiral_force(chir, m3, m4, mo, phi, E.params(tol=1e-12, max_iter=20000))
    ref = OF.force(lat, chir, m3, m4, mo, phi, tol=1e-12)
    assert info["true_rel_resid"] <= 1e-12
    assert np.abs(F.cpu().numpy() - ref).max() < 1e-9 * np.abs(ref).max()
