"""Python shim over the FP64 C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of bench.py, never by the product package.  It shares no code with
the HIP path; the only module both sides use is the seeded input generator.

All fields use the canonical layouts (complex128):
  links [Lt][Lz][Ly][Lx][mu][3][3], 4D [Lt][Lz][Ly][Lx][4][3], 5D [Ns][Lt][Lz][Ly][Lx][4][3].
``dims`` is (Lx, Ly, Lz, Lt) everywhere.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        P, I, D, L = C.c_void_p, C.c_int, C.c_double, C.c_long
        sig = {
            "or_gamma": (None, [I, P]),
            "or_hop": (None, [P, I, P, P, P, I]),
            "or_dw": (None, [P, I, D, P, P, P, I]),
            "or_mpm": (I, [I, P, D, I, P]),
            "or_k_omega": (I, [I, P, D, D, I, P, P, P]),
            "or_dt": (I, [P, I, D, I, P, D, D, P, P, P, I]),
            "or_ht": (I, [P, I, D, I, P, D, D, P, P, P]),
            "or_dodwf": (None, [P, I, D, I, P, D, D, P, P, P, I]),
            "or_ht_solve": (I, [P, I, D, I, P, D, D, P, P, P, D, I, P]),
            "or_dodwf_solve": (I, [P, I, D, I, P, D, D, P, P, P, D, I, P]),
            "or_chiral_action": (I, [P, I, D, I, P, I, D, D, D, P, P, P, D, I, P, P, P]),
            "or_hinv": (I, [P, I, D, I, P, D, D, P, P, P, D, I, P, P, P]),
            "or_at_inv": (I, [P, D, I, P, D, D, P, P, I, I]),
            "or_schur": (I, [P, I, D, I, P, D, D, P, P, P, I]),
            "or_dt_at": (I, [P, I, D, I, P, D, D, P, P, L, P, P, I]),
            "or_num_threads": (I, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _dims(dims):
    return np.ascontiguousarray(np.array(dims, dtype=np.int32))


class Lattice:
    """Holds the operator parameters: dims, links, m0, Ns, omega and the t boundary phase."""

    def __init__(self, dims, U, m0=1.3, Ns=None, omega=None, tbc=-1):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.U = _c128(U)
        assert self.U.size == self.V * 36
        self.m0 = float(m0)
        self.tbc = int(tbc)
        self.omega = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
        self.Ns = None if omega is None else len(self.omega)
        if Ns is not None:
            assert self.Ns == Ns
        self._L = _dims(self.dims)

    @property
    def shape4(self):
        Lx, Ly, Lz, Lt = self.dims
        return (Lt, Lz, Ly, Lx, 4, 3)

    @property
    def shape5(self):
        return (self.Ns,) + self.shape4

    # ---- 4D
    def hop(self, psi, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_hop(_p(self._L), self.tbc, _p(self.U), _p(psi), _p(out), int(dag))
        return out

    def dw(self, psi, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_dw(_p(self._L), self.tbc, self.m0, _p(self.U), _p(psi), _p(out), int(dag))
        return out

    # ---- s-space
    def mpm(self, m, chir):
        M = np.empty((self.Ns, self.Ns))
        lib().or_mpm(self.Ns, _p(self.omega), float(m), int(chir), _p(M))
        return M

    def k_omega(self, mj, mi, chir):
        k, rem = C.c_double(), C.c_double()
        Om = np.empty(self.Ns)
        lib().or_k_omega(self.Ns, _p(self.omega), float(mj), float(mi), int(chir), C.byref(k), _p(Om),
                         C.byref(rem))
        return k.value, Om, rem.value

    # ---- 5D
    def dt(self, psi, mp, mm, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_dt(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp), float(mm),
                    _p(self.U), _p(psi), _p(out), int(dag))
        return out

    def ht(self, psi, mp, mm):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_ht(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp), float(mm),
                    _p(self.U), _p(psi), _p(out))
        return out

    def dodwf(self, psi, mp, mm, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_dodwf(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp), float(mm),
                       _p(self.U), _p(psi), _p(out), int(dag))
        return out

    def at_inv(self, psi, mp, mm, parity=-1, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_at_inv(_p(self._L), self.m0, self.Ns, _p(self.omega), float(mp), float(mm), _p(psi),
                        _p(out), int(parity), int(dag))
        return out

    def schur(self, psi, mp, mm, dag=False):
        psi = _c128(psi)
        out = np.empty_like(psi)
        lib().or_schur(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp), float(mm),
                       _p(self.U), _p(psi), _p(out), int(dag))
        return out

    def dt_at(self, psi, mp, mm, sites, dag=False):
        psi = _c128(psi)
        sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
        out = np.empty((len(sites), self.Ns, 4, 3), dtype=np.complex128)
        lib().or_dt_at(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp), float(mm),
                       _p(self.U), _p(psi), len(sites), _p(sites), _p(out), int(dag))
        return out

    def ht_solve(self, b, mp, mm, tol=1e-10, maxit=100000):
        b = _c128(b)
        x = np.empty_like(b)
        rr = C.c_double()
        it = lib().or_ht_solve(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp),
                               float(mm), _p(self.U), _p(b), _p(x), float(tol), int(maxit), C.byref(rr))
        return x, it, rr.value

    def dodwf_solve(self, bp, mp, mm, tol=1e-10, maxit=100000):
        bp = _c128(bp)
        y = np.empty_like(bp)
        rr = C.c_double()
        it = lib().or_dodwf_solve(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mp),
                                  float(mm), _p(self.U), _p(bp), _p(y), float(tol), int(maxit), C.byref(rr))
        return y, it, rr.value

    def chiral_action(self, chir, m3, m4, mo, phi, tol=1e-10, maxit=100000):
        phi = _c128(phi)
        out = np.empty_like(phi)
        S, Si, rr = C.c_double(), C.c_double(), C.c_double()
        it = lib().or_chiral_action(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), int(chir),
                                    float(m3), float(m4), float(mo), _p(self.U), _p(phi), _p(out),
                                    float(tol), int(maxit), C.byref(S), C.byref(Si), C.byref(rr))
        return out, S.value, dict(iters=it, S_imag=Si.value, relres=rr.value)

    def hinv(self, phi, mlo, mhi, tol=1e-10, maxit=100000):
        phi = _c128(phi)
        out = np.empty_like(phi)
        S, Si = C.c_double(), C.c_double()
        rr = np.zeros(2)
        it = lib().or_hinv(_p(self._L), self.tbc, self.m0, self.Ns, _p(self.omega), float(mlo), float(mhi),
                           _p(self.U), _p(phi), _p(out), float(tol), int(maxit), C.byref(S), C.byref(Si),
                           _p(rr))
        return out, S.value, dict(iters=it, S_imag=Si.value, relres=tuple(rr))


def gamma(mu: int) -> np.ndarray:
    out = np.empty((4, 4), dtype=np.complex128)
    lib().or_gamma(int(mu), _p(out))
    return out


def parity_mask(dims) -> np.ndarray:
    """Boolean [Lt][Lz][Ly][Lx]: True on odd sites ((x+y+z+t) odd)."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    return ((x + y + z + t) & 1) == 1


def num_threads() -> int:
    return int(lib().or_num_threads())
