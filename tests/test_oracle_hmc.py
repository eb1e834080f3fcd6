"""Pins of the HMC oracle (oracle/hmc.py) against what the mathematics fixes: the unit field, gauge invariance,
finite differences of the action, the group manifold, reversibility and the second-order energy error of the
Omelyan integrator (Sec. I; Sec. III)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import hmc as H
from oracle import oracle as O


def _warm(rng, dims, amp):
    """Links exp(i amp X) with X random Hermitian traceless: a smooth field (small forces)."""
    Lx, Ly, Lz, Lt = dims
    P = rng.standard_normal((4, Lt, Lz, Ly, Lx, 8))
    U = np.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        X = H.algebra(P[mu]).reshape(-1, 3, 3)
        U[..., mu, :, :] = np.array([expm(1j * amp * x) for x in X]).reshape(Lt, Lz, Ly, Lx, 3, 3)
    return U


def test_unit_field_and_gauge_invariance():
    dims = (4, 2, 2, 4)
    Lx, Ly, Lz, Lt = dims
    one = np.broadcast_to(np.eye(3), (Lt, Lz, Ly, Lx, 4, 3, 3))
    assert abs(H.gauge_action(one, dims, 6.2)) < 1e-12
    assert np.abs(H.gauge_force(one, dims, 6.2)).max() < 1e-14
    rng = np.random.default_rng(1)
    U = H.random_su3(rng, (Lt, Lz, Ly, Lx, 4))
    S = H.gauge_action(U, dims, 6.2)
    g = H.random_su3(rng, (Lt, Lz, Ly, Lx))
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ H.dag(H.shift(g, mu))
    assert abs(H.gauge_action(Ug, dims, 6.2) - S) < 1e-10 * abs(S)
    # one link differs from 1: U_x at the origin closes 3 planes x 2 plaquettes, each with Re Tr U
    V = np.broadcast_to(np.eye(3, dtype=np.complex128), U.shape).copy()
    V[0, 0, 0, 0, 0] = U[0, 0, 0, 0, 0]
    ref = 6.2 * 6 * (1 - np.real(np.trace(U[0, 0, 0, 0, 0])) / 3)
    assert abs(H.gauge_action(V, dims, 6.2) - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 4, 3, 2)])
def test_gauge_force_is_the_derivative(dims):
    """Central finite differences of S_g along U_mu(x) -> exp(i w T^a) U_mu(x)."""
    rng = np.random.default_rng(2)
    Lx, Ly, Lz, Lt = dims
    U = H.random_su3(rng, (Lt, Lz, Ly, Lx, 4))
    beta = 5.7
    F = H.gauge_force(U, dims, beta)
    h = 1e-5
    sites = [(0, 0, 0, 0), (Lt - 1, Lz - 1, Ly - 1, Lx - 1), (1, 0, Ly - 1, 1)]
    for mu in range(4):
        for (t, z, y, x) in sites:
            for a in range(8):
                d = []
                for sg in (+1, -1):
                    V = U.copy()
                    V[t, z, y, x, mu] = expm(1j * sg * h * H.T[a]) @ U[t, z, y, x, mu]
                    d.append(H.gauge_action(V, dims, beta))
                fd = (d[0] - d[1]) / (2 * h)
                assert abs(fd - F[mu, t, z, y, x, a]) < 1e-6 * (1 + abs(fd)), (mu, t, z, y, x, a)


def test_omelyan_constant():
    """The minimum-norm coefficient of the second-order scheme, in closed form."""
    c = (2 * np.sqrt(326.0) + 36) ** (1 / 3)
    assert H.LAMBDA_OMELYAN == pytest.approx(0.5 - c / 12 + 1 / (6 * c), abs=1e-15)


def test_link_update_stays_in_su3():
    dims = (2, 2, 2, 4)
    rng = np.random.default_rng(3)
    U = H.random_su3(rng, (4, 2, 2, 2, 4))
    P = rng.standard_normal((4, 4, 2, 2, 2, 8))
    U1 = H.update_links(U, dims, P, 0.37)
    eye = np.eye(3)
    assert np.abs(H.dag(U1) @ U1 - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U1) - 1).max() < 1e-13
    # exp(i h P) exp(-i h P) = 1
    U2 = H.update_links(U1, dims, P, -0.37)
    assert np.abs(U2 - U).max() < 1e-13


def test_pure_gauge_md_is_reversible_and_second_order():
    dims = (4, 4, 2, 2)
    rng = np.random.default_rng(4)
    U = _warm(rng, dims, 0.4)
    P = rng.standard_normal((4, 2, 2, 4, 4, 8))
    sysm = H.System(dims, 5.7, 1.3, np.ones(4), [], [8])
    U1, P1, dH8, st = sysm.trajectory(U, P, tau=0.5)
    assert st["links"] == 16 and st["force"] == [24]
    U2, P2, _ = sysm.integrate(U1, -P1, 0.5)
    assert np.abs(U2 - U).max() < 1e-12 and np.abs(P2 + P).max() < 1e-11
    # second order: halving the step divides dH by 4 (5.5, 4.4, 4.1 from 4 steps on for this field)
    dH = [abs(H.System(dims, 5.7, 1.3, np.ones(4), [], [k]).trajectory(U, P, tau=0.5)[2]) for k in (8, 16, 32)]
    for a, b in zip(dH, dH[1:]):
        assert 3.6 < a / b < 4.6, dH
    assert dH[0] == pytest.approx(abs(dH8), rel=1e-12)


def _fermion_system(dims, steps, phi_seed=5):
    from paper_1710_09621_amd import inputs as IN
    rng = np.random.default_rng(phi_seed)
    Lx, Ly, Lz, Lt = dims
    omega = IN.optimal_omega(4)
    phis = [(rng.standard_normal((Lt, Lz, Ly, Lx, 4, 3)) + 1j * rng.standard_normal((Lt, Lz, Ly, Lx, 4, 3)))
            for _ in range(2)]
    # the new-MP splitting's middle and last actions at levels 1 and 2
    actions = [(1, +1, 0.05, 0.3, 1.0, phis[0]), (2, -1, 1.0, 0.3, 1.0, phis[1])]
    return H.System(dims, 5.7, IN.M0, omega, actions, steps)


def test_fermion_md_is_reversible_and_second_order():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(6)
    U = _warm(rng, dims, 0.3)
    P = rng.standard_normal((4, 4, 2, 2, 4, 8))
    sysm = _fermion_system(dims, [8, 2, 1])
    U1, P1, dH, st = sysm.trajectory(U, P, tau=0.25)
    assert st["force"] == [24, 6, 3] and st["links"] == 16
    U2, P2, _ = sysm.integrate(U1, -P1, 0.25)
    assert np.abs(U2 - U).max() < 1e-9 and np.abs(P2 + P).max() < 1e-8
    dHs = [abs(_fermion_system(dims, [4 * k, 2 * k, k]).trajectory(U, P, tau=0.5)[2]) for k in (1, 2)]
    assert 3.0 < dHs[0] / dHs[1] < 5.3, dHs


def test_fermion_force_matches_the_action():
    """The level force of a fermion level is the derivative of that level's actions (finite differences of
    the oracle's chiral actions along one link and generator)."""
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(7)
    U = _warm(rng, dims, 0.3)
    sysm = _fermion_system(dims, [4, 2, 1])
    sysm.actions = [a for a in sysm.actions if a[0] == 1]
    F = sysm.level_force(U, 1)
    h = 1e-5
    for (mu, t, z, y, x, a) in [(0, 0, 0, 0, 0, 3), (3, 3, 1, 1, 3, 7), (2, 1, 0, 1, 2, 0)]:
        d = []
        for sg in (+1, -1):
            V = U.copy()
            V[t, z, y, x, mu] = expm(1j * sg * h * H.T[a]) @ U[t, z, y, x, mu]
            d.append(sysm.fermion_action(V))
        fd = (d[0] - d[1]) / (2 * h)
        assert abs(fd - F[mu, t, z, y, x, a]) < 1e-6 * (1 + abs(fd))
