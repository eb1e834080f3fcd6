"""The mass-preconditioning splittings through the C ABI (one batch per splitting) against the oracle:
every chiral action of Eq.(noMP), of the old and the new cascade with two heavy masses (Eqs.(old_MP_N),
(new_MP_N)), equal to the oracle's at the solver tolerance."""
import pytest

from gpu_common import ctx_and_oracle, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    print("[gpu] mp splittings dims=(4, 4, 4, 4) Ns=8", flush=True)
    return ctx_and_oracle((4, 4, 4, 4), 8)


@pytest.mark.parametrize("kind,hs", [("none", []), ("old", [0.05, 0.3]), ("new", [0.05, 0.3])])
def test_splitting_actions(small, kind, hs):
    from paper_1710_09621_amd import eofa as E
    from paper_1710_09621_amd import inputs as IN
    from paper_1710_09621_amd import mpseq
    ctx, lat = small
    acts = mpseq.actions(kind, 0.01, hs, 1.0)
    phi = IN.gaussian_spinor(lat.shape4[:-2], 21)
    res = ctx.chiral_action_batch(acts, [phi] * len(acts), E.params(tol=1e-12, max_iter=20000))
    for a, r in zip(acts, res):
        ref, S, _ = lat.chiral_action(*a, phi, tol=1e-12)
        assert r.info[0]["true_rel_resid"] <= 1e-12, a
        assert relerr(r.out, ref) < 1e-9, a
        assert abs(r.S - S) < 1e-9 * abs(S), a
