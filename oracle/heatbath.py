"""Heat-bath generation of the EOFA pseudofermion fields (Sec. I, Eq.(CG_gaussian)).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.

Each chiral action of Eqs.(m1m2_m1m4) / (m1m2_m3m2) is S = phi^dag A phi with A a Hermitian positive-definite
operator on the 4D fields of one chirality c (out = A phi is Lattice.chiral_action).  Sec. I draws the
pseudofermion with weight exp(-S) from Gaussian noise eta of weight exp(-eta^dag eta) by solving
Eq.(CG_gaussian), (1/sqrt(H)) phi = eta with H^{-1} = A, i.e. phi = A^{-1/2} P_c eta.  For H^{-1}(m_j, m_i) of
Eq.(Hij), the - action on the P_- half plus the + action on the P_+ half, the two halves are independent:
phi = A_-^{-1/2} P_- eta + A_+^{-1/2} P_+ eta.

Two independent evaluations of A^{-1/2} eta:
* ``dense``: A as a matrix on the range of P_c, column by column from oracle chiral actions on unit vectors,
  and phi from its eigendecomposition (the definition; tiny lattices only);
* ``lanczos``: the Lanczos process on A started at P_c eta builds an orthonormal basis V_k and the tridiagonal
  T_k = V_k^dag A V_k; phi ~ |P_c eta| V_k T_k^{-1/2} e_1, stopped once two successive estimates agree to tol
  (one oracle chiral action per step, full reorthogonalisation).
"""
from __future__ import annotations

import numpy as np

from . import dense as Dn
from . import oracle as O


def chiral_projector(chir):
    g5 = O.gamma(4)
    return (np.eye(4) + chir * g5) / 2


def project(chir, phi):
    """P_c phi on a 4D field [..][4][3]."""
    return np.einsum("ab,...bc->...ac", chiral_projector(chir), phi)


def action_op(lat, chir, m3, m4, mo, tol=1e-13):
    """phi -> A phi of the chiral action (chir; m3, m4, mo as in Lattice.chiral_action)."""
    return lambda f: lat.chiral_action(chir, m3, m4, mo, f, tol=tol)[0]


def dense_block(lat, chir, m3, m4, mo, tol=1e-13):
    """(A restricted to range(P_c) as a matrix, basis B of that range) on a tiny lattice."""
    M = Dn.dense(action_op(lat, chir, m3, m4, mo, tol), lat.shape4)
    Pp, Pm = Dn.chiral_projectors(lat.V)
    P = Pp if chir > 0 else Pm
    w, v = np.linalg.eigh(P)
    B = v[:, w > 0.5]
    return B.conj().T @ M @ B, B


def dense_heatbath(lat, chir, m3, m4, mo, eta, tol=1e-13):
    """phi = A^{-1/2} P_c eta by the eigendecomposition of the dense A (the definition)."""
    A, B = dense_block(lat, chir, m3, m4, mo, tol)
    A = (A + A.conj().T) / 2
    w, v = np.linalg.eigh(A)
    x = B.conj().T @ np.asarray(eta).reshape(-1)
    y = v @ ((v.conj().T @ x) / np.sqrt(w))
    return (B @ y).reshape(lat.shape4), w


def lanczos_heatbath(lat, chir, m3, m4, mo, eta, tol=1e-12, kmax=60, solve_tol=1e-13):
    """phi = A^{-1/2} P_c eta from the Lanczos process on A (see the module docstring).  Returns (phi, steps)."""
    apply = action_op(lat, chir, m3, m4, mo, solve_tol)
    b = project(chir, np.asarray(eta, dtype=np.complex128))
    nb = np.linalg.norm(b)
    if nb == 0:
        return np.zeros_like(b), 0
    V = [b / nb]
    alpha, beta = [], []
    prev = None
    for k in range(kmax):
        w = project(chir, apply(V[-1]))
        a = np.vdot(V[-1], w).real
        alpha.append(a)
        for v in V:  # full reorthogonalisation
            w = w - np.vdot(v, w) * v
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        ev, Q = np.linalg.eigh(T)
        c = Q @ (Q[0, :] / np.sqrt(ev))  # T^{-1/2} e_1
        est = nb * sum(ci * vi for ci, vi in zip(c, V))
        if prev is not None and np.linalg.norm(est - prev) <= tol * np.linalg.norm(est):
            return est, k + 1
        prev = est
        bn = np.linalg.norm(w)
        if bn <= 1e-15 * nb:
            return est, k + 1
        beta.append(bn)
        V.append(w / bn)
    raise RuntimeError("Lanczos heat-bath did not converge")


def hinv_heatbath(lat, mlo, mhi, eta, tol=1e-12):
    """phi with weight exp(-phi^dag H^{-1}(m_hi, m_lo) phi) (Eq.(Hij)): the - action (m_lo,m_lo)/(m_lo,m_hi) on
    P_- eta and the + action (m_lo,m_hi)/(m_hi,m_hi) on P_+ eta."""
    pm, _ = lanczos_heatbath(lat, -1, mlo, mlo, mhi, eta, tol)
    pp, _ = lanczos_heatbath(lat, +1, mlo, mhi, mhi, eta, tol)
    return pm + pp
