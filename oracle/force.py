"""Oracle of the EOFA fermion force (test infrastructure only: imported by tests, never by the library).

For one chiral action (Sec. II, Eqs.(m1m2_m1m4), (m1m2_m3m2))
    S = phi^dag P [1 + c k Om^T H_T(m3, m4)^{-1} Om] P phi,   c = chirality, P = P_c,
the force on the link U_mu(x) is the derivative of S along U_mu(x) -> exp(i w^a T^a) U_mu(x), T^a = lambda^a / 2:
    dS/dw^a = -c k x^dag (dH_T/dw^a) x,    x = H_T^{-1} Om P phi,
since d(H^{-1}) = -H^{-1} dH H^{-1} and H_T is Hermitian.  With H_T = gamma_5 R_5 D_T and only the Wilson hop of
D_T depending on the links, x^dag dH_T x = y^dag dD_w x with y = gamma_5 R_5 x, and the link enters D_w once
forward (site x) and once backward (site x + mu).  Written out plainly here with numpy, for small lattices.
"""
import numpy as np

from . import oracle as O

# Gell-Mann matrices (SU(3) generators T^a = lambda^a / 2)
_LAM = np.zeros((8, 3, 3), dtype=np.complex128)
_LAM[0][0, 1] = _LAM[0][1, 0] = 1
_LAM[1][0, 1], _LAM[1][1, 0] = -1j, 1j
_LAM[2][0, 0], _LAM[2][1, 1] = 1, -1
_LAM[3][0, 2] = _LAM[3][2, 0] = 1
_LAM[4][0, 2], _LAM[4][2, 0] = -1j, 1j
_LAM[5][1, 2] = _LAM[5][2, 1] = 1
_LAM[6][1, 2], _LAM[6][2, 1] = -1j, 1j
_LAM[7] = np.diag([1, 1, -2]) / np.sqrt(3)
T = _LAM / 2


def action_parts(lat, chir, m3, m4, mo, phi, tol=1e-12):
    """(k, x): the mass factor k and the 5D solution x = H_T(m3, m4)^{-1} Om P phi of one chiral action."""
    k, Om, _ = lat.k_omega(mo, m4 if chir < 0 else m3, chir)
    g5 = O.gamma(4)
    P = (np.eye(4) + chir * g5) / 2
    Pphi = np.einsum("ab,...bc->...ac", P, np.asarray(phi, dtype=np.complex128))
    b = Om.reshape((-1,) + (1,) * Pphi.ndim) * Pphi[None]
    x = lat.ht_solve(b, m3, m4, tol=tol)
    x = x[0] if isinstance(x, tuple) else x
    return k, x


def force(lat, chir, m3, m4, mo, phi, tol=1e-12):
    """F[mu][t][z][y][x][a] = dS/dw^a for the link U_mu at that site (mu = 0..3 for x, y, z, t)."""
    k, x = action_parts(lat, chir, m3, m4, mo, phi, tol)
    g5 = O.gamma(4)
    y = np.einsum("ab,s...bc->s...ac", g5, x[::-1])           # y = gamma_5 R_5 x
    U = np.asarray(lat.U).reshape(lat.shape4[:4] + (4, 3, 3))  # [t][z][y][x][mu][3][3]
    Lt = lat.dims[3]
    F = np.zeros((4,) + lat.shape4[:4] + (8,))
    axis5 = {0: 4, 1: 3, 2: 2, 3: 1}  # field axis of direction mu in [s][t][z][y][x][spin][colour]
    for mu in range(4):
        g = O.gamma(mu)
        xf = np.roll(x, -1, axis=axis5[mu])                    # x(z + mu)
        yf = np.roll(y, -1, axis=axis5[mu])
        Um = U[..., mu, :, :]
        # term 1: y(z)^dag (1 - g) T^a U x(z + mu); term 2: y(z + mu)^dag (1 + g) U^dag T^a x(z)
        v = np.einsum("ab,s...bc->s...ac", np.eye(4) - g, xf)
        w = np.einsum("ab,s...bc->s...ac", np.eye(4) + g, x)
        B1 = np.einsum("s...ai,s...aj->...ij", v, y.conj())    # B1[c'][c] = sum v[c'] conj(y[c])
        B2 = np.einsum("s...ai,s...aj->...ij", w, yf.conj())
        M = Um @ B1 - B2 @ np.conj(np.swapaxes(Um, -1, -2))
        if lat.tbc != 1 and mu == 3:                           # the boundary phase of the links t = Lt - 1 -> 0
            M[Lt - 1] *= lat.tbc
        tr = np.einsum("aij,...ji->...a", T, M)                # Tr[T^a M]
        F[mu] = -(chir * k / 2) * np.imag(tr)                 # Re(i (c k / 2) Tr[T^a M])
    return F
