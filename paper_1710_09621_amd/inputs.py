"""Seeded synthetic inputs: gauge links, Gaussian sources and R5-symmetric weights.

This module is shared by the FP64 oracle and the HIP path and holds none of the
operator arithmetic: it only draws random numbers and evaluates the input
conventions below.

* Links follow the parametrisation U = exp(i A^a t^a) of Sec. I (t^a = lambda^a / 2,
  Gell-Mann matrices) with A^a = eps * theta_a, theta_a ~ N(0, 1) i.i.d. ("near-unit"
  links; eps sets the roughness).  Draw order: site lexicographic (x fastest, t
  slowest), then mu = x, y, z, t, then a = 1..8.
* Sources have the weight exp(-eta^dagger eta) of Sec. I: real and imaginary parts
  i.i.d. N(0, 1/2).  Draw order: site, spin, colour, then (re, im).
* The weights omega_s of the optimal DWF with R5 symmetry (Sec. III.A names them but
  gives no formula): the Ns/2 distinct values solve the minimax problem
  min max_{x in [lmin, lmax]} prod_j |(1 - w_j x) / (1 + w_j x)|, whose solution is
  Zolotarev's, w_j = 1 / (lmax * dn((2j-1) K(k') / Ns, k')), k' = sqrt(1 - (lmin/lmax)^2);
  each value appears twice, arranged so that omega_s = omega_{Ns+1-s}.

Canonical layouts (complex128):
  links   [Lt][Lz][Ly][Lx][mu][3][3]      (row, column)
  4D spinor [Lt][Lz][Ly][Lx][spin][colour]
  5D spinor [Ns][Lt][Lz][Ly][Lx][spin][colour]
"""
from __future__ import annotations

import numpy as np

__all__ = ["gell_mann", "gauge_links", "unit_links", "gaussian_spinor", "optimal_omega",
           "random_su3", "CONFIGS"]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda^a, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    return lam


def _exp_i_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a stack of Hermitian 3x3 matrices via the eigen-decomposition,
    followed by one SU(3) projection (fix the determinant phase)."""
    w, v = np.linalg.eigh(h)
    u = np.einsum("nij,nj,nkj->nik", v, np.exp(1j * w), v.conj(), optimize=True)
    # h is traceless so det u = 1 up to rounding; remove the residual phase.
    det = np.linalg.det(u)
    u *= (det.conj() / np.abs(det))[:, None, None] ** (1.0 / 3.0)
    return u


def gauge_links(dims, eps: float, seed: int, chunk: int = 1 << 20) -> np.ndarray:
    """Near-unit SU(3) links U_mu(x) = exp(i eps theta_a t^a), canonical layout.

    dims = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    n = Lx * Ly * Lz * Lt * 4
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = gell_mann() / 2.0
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for start in range(0, n, chunk):
        stop = min(n, start + chunk)
        theta = rng.standard_normal((stop - start, 8))
        h = eps * np.einsum("na,aij->nij", theta, gen, optimize=True)
        out[start:stop] = _exp_i_hermitian(h)
    return out.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def unit_links(dims) -> np.ndarray:
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    u = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3(n: int, seed: int) -> np.ndarray:
    """Haar-like random SU(3) matrices (QR of a complex Gaussian), shape (n, 3, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q *= (det.conj() / np.abs(det))[:, None, None] ** (1.0 / 3.0)
    return q


def gaussian_spinor(shape, seed: int) -> np.ndarray:
    """Complex Gaussian field with weight exp(-eta^dagger eta): shape + (4, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    full = tuple(shape) + (4, 3, 2)
    g = rng.standard_normal(full) * np.sqrt(0.5)
    return g[..., 0] + 1j * g[..., 1]


def optimal_omega(Ns: int, lmin: float = 0.05, lmax: float = 6.2) -> np.ndarray:
    """R5-symmetric optimal weights omega_s, s = 1..Ns (Ns even)."""
    from scipy.special import ellipj, ellipk
    if Ns % 2:
        raise ValueError("Ns must be even")
    n = Ns // 2
    kp2 = 1.0 - (lmin / lmax) ** 2
    K = ellipk(kp2)
    p = np.array([lmax * ellipj((2 * j - 1) * K / (2 * n), kp2)[2] for j in range(1, n + 1)])
    w = 1.0 / p  # ascending
    return np.concatenate([w, w[::-1]])


def cnn_params(seed, scale=1.0):
    """Seeded parameters of the 4-layer preconditioner network (channels 24, 32, 32, 32, 24, 81 taps):
    per layer N(0, scale^2 / (81 cin)) weights [81][32 out][32 in], N(0, (0.1 scale)^2) biases [32],
    zero in the padding channels.  Returns float32 [4 * (81 * 1024 + 32)]."""
    cin, cout = (24, 32, 32, 32), (32, 32, 32, 24)
    wsz, lsz = 81 * 32 * 32, 81 * 32 * 32 + 32
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(4 * lsz)
    for l in range(4):
        W = p[l * lsz: l * lsz + wsz].reshape(81, 32, 32)
        W[:, :cout[l], :cin[l]] = rng.normal(0, scale / np.sqrt(81 * cin[l]), (81, cout[l], cin[l]))
        p[l * lsz + wsz: l * lsz + wsz + cout[l]] = rng.normal(0, 0.1 * scale, cout[l])
    return p.astype(np.float32)


# The five synthetic workloads (lattice dims are (Lx, Ly, Lz, Lt)).
CONFIGS = {
    1: dict(dims=(4, 4, 4, 4), Ns=8, eps=0.3, seed=1, masses=(0.05, 1.0), nsrc=1),
    2: dict(dims=(16, 16, 16, 32), Ns=16, eps=0.5, seed=2, masses=(0.01, 0.1), nsrc=4),
    3: dict(dims=(24, 24, 24, 48), Ns=16, eps=0.6, seed=3,
            pairs=((0.005, 0.05), (0.05, 0.2), (0.2, 1.0)), nsrc=4),
    4: dict(dims=(16, 16, 16, 32), Ns=16, eps=0.5, seed=4, masses=(0.01, 0.1),
            train_seeds=tuple(range(40, 48)), heldout_seeds=(48, 49)),
    5: dict(dims=(32, 32, 32, 64), Ns=16, eps=0.7, seed=5, masses=(0.01, 0.1, 1.0), nsrc=8),
}
M0 = 1.3
