"""Oracle of the HMC molecular dynamics of one-flavour EOFA (Sec. I and Sec. III).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.

Phase space: the links U_mu(x) in SU(3) (canonical layout [t][z][y][x][mu][3][3], periodic) and their momenta
P_mu(x) = sum_a P^a T^a, T^a = lambda^a / 2, stored as the 8 real components P[mu][t][z][y][x][a].  Sec. I:
    H = 1/2 sum P^a P^a + S_g(U) + sum_i S_i(U),
    dU/dtau = i P U,    dP^a/dtau = -dH/dw^a   (derivative along U -> exp(i w^a T^a) U),
with S_g the Wilson plaquette action (Sec. III uses it at beta = 6.20)
    S_g = beta sum_{x, mu < nu} (1 - Re Tr U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag / 3)
and S_i = phi_i^dag A_i phi_i the chiral actions of an EOFA splitting (their forces: oracle.force).

Integrator (Sec. III): the second-order minimum-norm (Omelyan) scheme, nested over time scales as in the
multiple-time-scale method.  Level 0 holds the gauge action, level j >= 1 a set of fermion actions.  With
k_j the total number of steps of level j per trajectory of length tau (k_0 >= k_1 >= ...), one step of level j
of size e = tau / k_j is
    P += -lam e F_j;  X_{j-1}(e / 2);  P += -(1 - 2 lam) e F_j;  X_{j-1}(e / 2);  P += -lam e F_j,
where X_{j-1}(h) runs k_{j-1} / (2 k_j) steps of level j - 1 over time h, and X_{-1}(h) is the link update
U <- exp(i h P) U.  Adjacent momentum updates of one level are applied separately (no merging), which is
the same map up to rounding.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import force as Fo
from . import oracle as O

LAMBDA_OMELYAN = 0.1931833275037836
T = Fo.T  # generators lambda^a / 2


def links(U, dims):
    """U as [t][z][y][x][mu][3][3]."""
    Lx, Ly, Lz, Lt = dims
    return np.asarray(U, dtype=np.complex128).reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # array axis of direction mu in [t][z][y][x]


def shift(a, mu, n=1):
    """a(x + n mu) as an array over x (periodic)."""
    return np.roll(a, -n, axis=_AXIS[mu])


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def plaquette(U, dims, mu, nu):
    """U_mu nu(x) = U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag at every x."""
    U = links(U, dims)
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]
    return Um @ shift(Un, mu) @ dag(shift(Um, nu)) @ dag(Un)


def gauge_action(U, dims, beta):
    """S_g, the definition above (6 planes per site)."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s += np.sum(1.0 - np.real(np.trace(plaquette(U, dims, mu, nu), axis1=-2, axis2=-1)) / 3.0)
    return beta * s


def mean_plaquette(U, dims):
    """Average of Re Tr U_mu nu / 3 over sites and planes."""
    V = int(np.prod(dims))
    return 1.0 - gauge_action(U, dims, 1.0) / (6 * V)


def staples(U, dims, mu):
    """Sum over nu != mu of the staples A such that the plaquettes holding U_mu(x) are Tr(U_mu(x) A)."""
    U = links(U, dims)
    Um = U[..., mu, :, :]
    A = np.zeros_like(Um)
    for nu in range(4):
        if nu == mu:
            continue
        Un = U[..., nu, :, :]
        # U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag
        A += shift(Un, mu) @ dag(shift(Um, nu)) @ dag(Un)
        # U_mu(x) U_nu(x + mu - nu)^dag U_mu(x - nu)^dag U_nu(x - nu): the plaquette (mu, nu) at x - nu
        Un_m = shift(Un, nu, -1)
        A += dag(shift(shift(Un, mu), nu, -1)) @ dag(shift(Um, nu, -1)) @ Un_m
    return A


def gauge_force(U, dims, beta):
    """F[mu][t][z][y][x][a] = dS_g/dw^a along U_mu(x) -> exp(i w^a T^a) U_mu(x).

    The link enters S_g as -(beta / 3) Re Tr(U A) with A its staple sum, so the derivative is
    -(beta / 3) Re Tr(i T^a U A) = (beta / 3) Im Tr(T^a U A).
    """
    U6 = links(U, dims)
    F = np.zeros((4,) + U6.shape[:4] + (8,))
    for mu in range(4):
        M = U6[..., mu, :, :] @ staples(U, dims, mu)
        F[mu] = (beta / 3.0) * np.imag(np.einsum("aij,...ji->...a", T, M))
    return F


def algebra(P):
    """sum_a P^a T^a for P[...][8]."""
    return np.einsum("...a,aij->...ij", P, T)


def kinetic(P):
    return 0.5 * float(np.sum(np.asarray(P) ** 2))


def update_links(U, dims, P, h):
    """U_mu(x) <- exp(i h P_mu(x)) U_mu(x) (matrix exponential of the library)."""
    U6 = links(U, dims).copy()
    for mu in range(4):
        X = 1j * h * algebra(P[mu])
        E = np.empty_like(X)
        flatX, flatE = X.reshape(-1, 3, 3), E.reshape(-1, 3, 3)
        for i in range(flatX.shape[0]):
            flatE[i] = expm(flatX[i])
        U6[..., mu, :, :] = E @ U6[..., mu, :, :]
    return U6


def force_to_mu_first(F, dims):
    """oracle.force's F[mu][t][z][y][x][a] is already in this layout; kept for symmetry."""
    return np.asarray(F).reshape((4,) + tuple(reversed(dims)) + (8,))


class System:
    """The HMC system: gauge coupling, the fermion operator parameters and the actions of each level.

    actions: list of (level, chir, m3, m4, mo, phi) with level >= 1; steps: [k_0, k_1, ...] total steps per
    trajectory of each level.
    """

    def __init__(self, dims, beta, m0, omega, actions, steps, tbc=-1, tol=1e-12):
        self.dims, self.beta, self.m0, self.omega = tuple(dims), float(beta), float(m0), np.asarray(omega)
        self.actions, self.steps, self.tbc, self.tol = list(actions), list(steps), tbc, tol
        for a in self.actions:
            assert 1 <= a[0] < len(self.steps)
        for j in range(1, len(self.steps)):
            assert self.steps[j - 1] % (2 * self.steps[j]) == 0, "k_{j-1} must be a multiple of 2 k_j"

    def lattice(self, U):
        return O.Lattice(self.dims, links(U, self.dims).reshape(-1), self.m0, omega=self.omega, tbc=self.tbc)

    def fermion_action(self, U):
        lat = self.lattice(U)
        return sum(lat.chiral_action(c, m3, m4, mo, phi, tol=self.tol)[1] for _, c, m3, m4, mo, phi in self.actions)

    def hamiltonian(self, U, P):
        return kinetic(P) + gauge_action(U, self.dims, self.beta) + self.fermion_action(U)

    def level_force(self, U, j):
        if j == 0:
            return gauge_force(U, self.dims, self.beta)
        lat = self.lattice(U)
        F = 0.0
        for lev, c, m3, m4, mo, phi in self.actions:
            if lev == j:
                F = F + Fo.force(lat, c, m3, m4, mo, phi, tol=self.tol)
        return F

    def integrate(self, U, P, tau, level=None, stats=None):
        """Run the nested Omelyan integration of length tau from level `level` (default: the outermost)."""
        if level is None:
            level = len(self.steps) - 1
        if stats is None:
            stats = {"force": [0] * len(self.steps), "links": 0}
        n = self.steps[level] if level == len(self.steps) - 1 else self.steps[level] // (2 * self.steps[level + 1])
        e = tau / n
        lam = LAMBDA_OMELYAN

        def inner(U, P, h):
            if level == 0:
                stats["links"] += 1
                return update_links(U, self.dims, P, h), P
            return self.integrate(U, P, h, level - 1, stats)[:2]

        def kick(U, P, h):
            stats["force"][level] += 1
            return P - h * self.level_force(U, level)

        for _ in range(n):
            P = kick(U, P, lam * e)
            U, P = inner(U, P, e / 2)
            P = kick(U, P, (1 - 2 * lam) * e)
            U, P = inner(U, P, e / 2)
            P = kick(U, P, lam * e)
        return U, P, stats

    def trajectory(self, U, P, tau=1.0):
        """(U', P', dH, stats): the molecular dynamics of Sec. I, step (5), and dH = H(U', P') - H(U, P)."""
        H0 = self.hamiltonian(U, P)
        U1, P1, stats = self.integrate(links(U, self.dims), np.asarray(P, dtype=np.float64), tau)
        H1 = self.hamiltonian(U1, P1)
        return U1, P1, H1 - H0, stats


def random_su3(rng, shape):
    """Haar-like random SU(3) matrices (QR of complex Gaussians, phases fixed, det made 1)."""
    Z = (rng.standard_normal(shape + (3, 3)) + 1j * rng.standard_normal(shape + (3, 3))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[..., None, None]
