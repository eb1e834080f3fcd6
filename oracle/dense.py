"""Dense brute-force companions of the oracle for tiny lattices (2^4, small Ns).

TEST INFRASTRUCTURE ONLY.  Builds dense matrices column by column from the C oracle's
operator applications and evaluates the paper's determinant statements with LAPACK
(slogdet / solve / eigvalsh), plus the free-field closed forms used as pins.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def dense(apply, shape):
    """Dense matrix of a linear map given as apply(field)->field of the given shape."""
    n = int(np.prod(shape))
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shape)).reshape(n)
        e[j] = 0.0
    return M


def chiral_projectors(nsites: int, ns: int = 1):
    """P_+ and P_- as dense matrices on fields [ns][nsites][4][3] (gamma_5 from the oracle)."""
    g5 = O.gamma(4)
    Pp = (np.eye(4) + g5) / 2
    Pm = (np.eye(4) - g5) / 2
    I3 = np.eye(3)
    return (np.kron(np.eye(ns * nsites), np.kron(Pp, I3)), np.kron(np.eye(ns * nsites), np.kron(Pm, I3)))


def omega_embed(lat: "O.Lattice", Om: np.ndarray):
    """The 5D <- 4D map phi -> Om_s phi as a dense matrix."""
    return np.kron(Om.reshape(-1, 1), np.eye(lat.V * 12))


def logdet(M):
    sign, la = np.linalg.slogdet(M)
    return la, sign


def subspace_logdet(M, P):
    """log|det| and phase of M restricted to the range of the projector P."""
    w, v = np.linalg.eigh((P + P.conj().T) / 2)
    B = v[:, w > 0.5]
    return logdet(B.conj().T @ M @ B)


def free_dw_momentum(p, m0):
    """Closed form of the free (U = 1) Wilson operator on a plane wave e^{ip.x}:
    D_w(p) = (4 - m0 - sum_mu cos p_mu) + i sum_mu gamma_mu sin p_mu."""
    out = (4.0 - m0 - np.sum(np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        out = out + 1j * np.sin(p[mu]) * O.gamma(mu)
    return out


def overlap_logdet(Dw_dense, g5_dense, omega, m):
    """log det of the Zolotarev-type overlap operator that the optimal DWF reproduces:
    D_ov(m) = (1+m)/2 + (1-m)/2 gamma_5 S(H_w),  H_w = gamma_5 D_w,
    S = (1 - prod_s T_s) (1 + prod_s T_s)^{-1},  T_s = (1 - omega_s H_w)(1 + omega_s H_w)^{-1}."""
    Hw = g5_dense @ Dw_dense
    n = Hw.shape[0]
    I = np.eye(n)
    T = I.copy()
    for w in omega:
        T = T @ np.linalg.solve(I + w * Hw, I - w * Hw)
    S = (I - T) @ np.linalg.inv(I + T)
    D = (1 + m) / 2 * I + (1 - m) / 2 * g5_dense @ S
    return logdet(D)
