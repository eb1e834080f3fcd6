"""Heat-bath pseudofermions on the GPU (Sec. I, Eq.(CG_gaussian)) against the oracle's Lanczos evaluation of
A^{-1/2} P_c eta, itself pinned to the dense definition (tests/test_oracle_heatbath.py).  The bar: the rational
approximation is asked for 1e-12 and every shifted solve reaches a true residual of 1e-10, so the GPU field must
agree with the oracle's (Lanczos to 1e-12, solves to 1e-13) to 1e-8 relative to its largest component."""
import numpy as np
import pytest
import torch

from gpu_common import ctx_and_oracle
from oracle import heatbath as HB
from paper_1710_09621_amd import inputs as IN

pytestmark = pytest.mark.gpu

# the three actions of Eq.(new_MP) with (m, m_h, M) = (0.01, 0.1, 1.0) at Ns = 8; at Ns = 16 (the lane-exchange
# path of the kernels) two actions on a small lattice with heavier masses, where the oracle's unpreconditioned
# solves stay short
CASES = [((4, 4, 4, 4), 8, (-1, 0.01, 0.01, 0.1)), ((4, 4, 4, 4), 8, (+1, 0.01, 0.1, 1.0)),
         ((4, 4, 4, 4), 8, (-1, 1.0, 0.1, 1.0)), ((2, 2, 2, 4), 16, (-1, 0.05, 0.05, 0.5)),
         ((2, 2, 2, 4), 16, (+1, 0.05, 0.5, 1.0))]


@pytest.mark.parametrize("dims,Ns,act", CASES, ids=lambda c: str(c))
def test_chiral_heatbath_matches_oracle(dims, Ns, act):
    from paper_1710_09621_amd import eofa as E
    print(f"[gpu] chiral heat-bath dims={dims} Ns={Ns} action {act}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns, eps=0.7, seed=95)
    eta = IN.gaussian_spinor(lat.shape4[:-2], 96)
    phi, info = ctx.chiral_heatbath(*act, torch.as_tensor(eta), rel_err=1e-12, verify=True,
                                    p=E.params(tol=1e-10))
    ref, steps = HB.lanczos_heatbath(lat, *act, eta, tol=1e-12)
    got = phi.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  poles {info['npoles']} (approx err {info['approx_err']:.1e} on [{info['lo']:.3f}, {info['hi']:.3f}]), "
          f"solves {info['iters_max']} iters / resid {info['true_rel_resid_max']:.1e}, check {info['check']:.1e}; "
          f"oracle Lanczos steps {steps}; max rel diff {err:.2e}")
    assert err < 1e-8
    assert abs(info["check"]) < 1e-8 and info["true_rel_resid_max"] <= 1e-10
    assert np.all(HB.project(-act[0], got) == 0)  # the other chiral half is zero


def test_full_heatbath_matches_oracle():
    from paper_1710_09621_amd import eofa as E
    dims, Ns = (4, 4, 4, 4), 8
    print(f"[gpu] heat-bath of H^-1(m_hi, m_lo) dims={dims} Ns={Ns}", flush=True)
    ctx, lat = ctx_and_oracle(dims, Ns, eps=0.7, seed=97)
    eta = IN.gaussian_spinor(lat.shape4[:-2], 98)
    for prec in (E.FP64, E.MIXED_FP16):
        phi, info = ctx.heatbath(torch.as_tensor(eta), 0.05, 1.0, rel_err=1e-12, verify=True,
                                 p=E.params(tol=1e-10, prec=prec))
        ref = HB.hinv_heatbath(lat, 0.05, 1.0, eta, tol=1e-12)
        err = np.abs(phi.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"  prec {prec}: max rel diff {err:.2e}, checks {[i['check'] for i in info]}")
        assert err < 1e-8 and all(abs(i["check"]) < 1e-8 for i in info)
    # the action of the generated field is the noise norm: S(phi) = phi^dag H^{-1} phi = |eta|^2
    r = ctx.hinv(phi, 0.05, 1.0, E.params(tol=1e-12))
    assert abs(r.S / float(np.vdot(eta, eta).real) - 1) < 1e-9


def test_equal_masses_return_the_projected_noise():
    from paper_1710_09621_amd import eofa as E
    ctx, lat = ctx_and_oracle((4, 4, 4, 4), 8)
    eta = IN.gaussian_spinor(lat.shape4[:-2], 99)
    phi, info = ctx.chiral_heatbath(-1, 0.2, 0.2, 0.2, torch.as_tensor(eta))
    assert info["npoles"] == 0
    assert np.array_equal(phi.cpu().numpy(), HB.project(-1, eta))


@pytest.mark.parametrize("bad", [dict(rel_err=0.0), dict(rel_err=1e-30), dict(lo=1.0, hi=0.5)])
def test_heatbath_bad_arguments_are_einval(bad):
    from paper_1710_09621_amd import eofa as E
    ctx, lat = ctx_and_oracle((4, 4, 4, 4), 8)
    eta = torch.as_tensor(IN.gaussian_spinor(lat.shape4[:-2], 100))
    with pytest.raises(E.EofaError) as ei:
        ctx.chiral_heatbath(-1, 0.01, 0.01, 0.1, eta, **bad)
    assert ei.value.status == E.EINVAL
