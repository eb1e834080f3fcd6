"""Python binding of the gfx950 EOFA library (libeofa.so) over its C ABI.

Argument marshalling only: every step of the solve runs in the HIP library.  Torch
supplies device memory and the stream.  There is no CPU fallback: if the library is
missing or no GPU is visible, every call raises.

Canonical layouts (torch.complex128 on the GPU), dims = (Lx, Ly, Lz, Lt):
  links (Lt, Lz, Ly, Lx, 4, 3, 3); 4D (Lt, Lz, Ly, Lx, 4, 3); 5D (Ns, Lt, Lz, Ly, Lx, 4, 3).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EOFA_LIB") or os.path.join(_HERE, "libeofa.so")
_lib = None

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESTATE, ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED_FP32, MIXED_FP16 = 0, 1, 2
PC_NONE, PC_LEARNED = 0, 1
CNN_NPARAM = 4 * (81 * 32 * 32 + 32)
HB_BATCH = 8  # the heat-bath's shifted solves run as one multi-RHS batch of at most 8 systems
OPS = dict(DW=0, HOP=1, DT=2, DT_DAG=3, HT=4, AT_INV=5, SCHUR=6, SCHUR_DAG=7, SCHUR_NORMAL=8, DODWF=9, DODWF_DAG=10,
           HOP_EO=11, HOP_OE=12)
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV", -5: "ESTATE", -6: "ENOTIMPL"}


class EofaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("prec", C.c_int), ("pc", C.c_int),
                ("reliable_delta", C.c_double), ("use_graph", C.c_int), ("check_every", C.c_int)]


NKERN = 5
KERNELS = ("hop", "schur_w", "hop_dag", "schur_q", "xp")  # K1 .. K5 of one FP64 CG iteration


class KernelStats(C.Structure):
    _fields_ = [("ms", C.c_double * NKERN), ("launches", C.c_long * NKERN), ("bytes", C.c_double * NKERN)]


class HeatbathInfo(C.Structure):
    _fields_ = [("npoles", C.c_int), ("approx_err", C.c_double), ("lo", C.c_double), ("hi", C.c_double),
                ("check", C.c_double), ("iters_max", C.c_int), ("true_rel_resid_max", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("op_applies", C.c_int), ("reliable_updates", C.c_int),
                ("fell_back", C.c_int), ("true_rel_resid", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MdAction(C.Structure):
    _fields_ = [("chir", C.c_int), ("m3", C.c_double), ("m4", C.c_double), ("mo", C.c_double), ("level", C.c_int),
                ("phi", C.c_void_p)]


class MdParams(C.Structure):
    _fields_ = [("beta", C.c_double), ("tau", C.c_double), ("nlevels", C.c_int), ("steps", C.c_int * 4),
                ("metropolis_u", C.c_double), ("chrono", C.c_int), ("force_tol", C.c_double)]


class MdInfo(C.Structure):
    _fields_ = [("H0", C.c_double), ("H1", C.c_double), ("dH", C.c_double), ("K0", C.c_double),
                ("K1", C.c_double), ("Sg0", C.c_double), ("Sg1", C.c_double), ("Sf0", C.c_double),
                ("Sf1", C.c_double), ("accepted", C.c_int), ("force_evals", C.c_int * 4), ("link_updates", C.c_int),
                ("cg_iters", C.c_long), ("seconds", C.c_double), ("force_max", C.c_double * 8),
                ("force_mean", C.c_double * 8), ("gauge_force0", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("force_evals", "force_max", "force_mean"):
            d[k] = list(getattr(self, k))
        return d


def params(tol=1e-10, max_iter=100000, prec=FP64, pc=PC_NONE, reliable_delta=0.0, use_graph=0, check_every=0):
    return SolveParams(tol, max_iter, prec, pc, reliable_delta, use_graph, check_every)


def load():
    """Load libeofa.so (built beforehand by build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1710_09621_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P, I, D, Z = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    PP = C.POINTER(C.c_void_p)
    sig = {
        "eofa_create": [C.POINTER(C.c_void_p), C.POINTER(C.c_int), I, D, C.POINTER(C.c_double), I, P],
        "eofa_workspace_size": [P, C.POINTER(SolveParams), I, C.POINTER(C.c_size_t)],
        "eofa_set_workspace": [P, P, Z],
        "eofa_set_gauge": [P, P],
        "eofa_hinv": [P, D, D, P, P, C.POINTER(C.c_double), C.POINTER(SolveParams), C.POINTER(SolveInfo)],
        "eofa_chiral_action": [P, I, D, D, D, P, P, C.POINTER(C.c_double), C.POINTER(SolveParams),
                               C.POINTER(SolveInfo)],
        "eofa_chiral_force": [P, I, D, D, D, P, P, C.POINTER(C.c_double), C.POINTER(SolveParams),
                              C.POINTER(SolveInfo)],
        "eofa_chiral_action_batch": [P, I, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), PP, PP, C.POINTER(C.c_double),
                                     C.POINTER(SolveParams), C.POINTER(SolveInfo)],
        "eofa_hinv_batch": [P, I, C.POINTER(C.c_double), C.POINTER(C.c_double), PP, PP, C.POINTER(C.c_double),
                            C.POINTER(SolveParams), C.POINTER(SolveInfo)],
        "eofa_solve_ht": [P, D, D, P, P, C.POINTER(SolveParams), C.POINTER(SolveInfo)],
        "eofa_chiral_heatbath": [P, I, D, D, D, P, P, D, D, D, I, C.POINTER(SolveParams), C.POINTER(HeatbathInfo)],
        "eofa_heatbath": [P, D, D, P, P, D, I, C.POINTER(SolveParams), C.POINTER(HeatbathInfo)],
        "eofa_inv_sqrt_rational": [D, D, I, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)],
        "eofa_solve_ht_batch": [P, I, C.POINTER(C.c_double), C.POINTER(C.c_double), PP, PP, C.POINTER(SolveParams),
                                C.POINTER(SolveInfo)],
        "eofa_apply": [P, I, D, D, P, P, I],
        "eofa_apply_static": [P, I, D, D, P, P, I],
        "eofa_kernel_timing": [P, I, I, C.POINTER(KernelStats)],
        "eofa_cg_block": [P, I, D, D, P, I, C.POINTER(C.c_double)],
        "eofa_set_precond": [P, C.POINTER(C.c_float), Z, I],
        "eofa_graph_stats": [P, C.POINTER(C.c_long), C.POINTER(C.c_int)],
        "eofa_cnn_init": [P, C.c_ulonglong, I],
        "eofa_cnn_params": [P, C.POINTER(C.c_float), Z],
        "eofa_cnn_apply": [P, P, P],
        "eofa_cnn_train_step": [P, P, P, D, C.POINTER(C.c_double), C.POINTER(C.c_float)],
        "eofa_training_pairs": [P, D, D, C.c_ulonglong, I, PP, PP, C.POINTER(C.c_int)],
        "eofa_dslash_bench": [P, I, I, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "eofa_autotune": [P, I, I, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "eofa_set_schedule": [P, I, C.POINTER(C.c_int)],
        "eofa_schedule_candidates": [P, I, I, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "eofa_gauge_action": [P, P, D, C.POINTER(C.c_double)],
        "eofa_gauge_force": [P, P, D, P],
        "eofa_md_trajectory": [P, P, P, I, C.POINTER(MdAction), C.POINTER(MdParams), C.POINTER(SolveParams),
                               C.POINTER(MdInfo)],
        "eofa_last_error": [P],
        "eofa_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.eofa_last_error.restype = C.c_char_p
    lib.eofa_destroy.restype = None
    _lib = lib
    return lib


def exported_symbols():
    """Names the library exports (for the ABI test)."""
    lib = load()
    return [n for n in ("eofa_create", "eofa_workspace_size", "eofa_set_workspace", "eofa_set_gauge", "eofa_hinv",
                        "eofa_chiral_action", "eofa_chiral_force", "eofa_chiral_action_batch", "eofa_hinv_batch", "eofa_solve_ht", "eofa_solve_ht_batch", "eofa_chiral_heatbath", "eofa_heatbath",
                        "eofa_inv_sqrt_rational", "eofa_schedule_candidates",
                        "eofa_gauge_action", "eofa_gauge_force", "eofa_md_trajectory",
                        "eofa_apply", "eofa_apply_static", "eofa_dslash_bench", "eofa_autotune", "eofa_set_schedule", "eofa_cnn_init",
                        "eofa_cnn_params", "eofa_cnn_apply", "eofa_cnn_train_step", "eofa_training_pairs",
                        "eofa_kernel_timing", "eofa_cg_block", "eofa_graph_stats", "eofa_set_precond",
                        "eofa_last_error", "eofa_destroy") if hasattr(lib, n)]


def inv_sqrt_rational(lo, hi, n):
    """The heat-bath's rational approximation of x^{-1/2} on [lo, hi] with n poles (host only):
    (a0, a[n], b[n], err) with x^{-1/2} ~ a0 + sum a_l / (x + b_l)."""
    lib = load()
    a0, err = C.c_double(), C.c_double()
    a, b = (C.c_double * n)(), (C.c_double * n)()
    st = lib.eofa_inv_sqrt_rational(float(lo), float(hi), int(n), C.byref(a0), a, b, C.byref(err))
    if st != OK:
        raise EofaError(st, "eofa_inv_sqrt_rational")
    return a0.value, np.array(a[:]), np.array(b[:]), err.value


def _ptr(t):
    return C.c_void_p(t.data_ptr())


@dataclass
class Result:
    out: object
    S: float
    info: list


class Context:
    """One lattice + weights + stream.  Not thread-safe."""

    def __init__(self, dims, Ns, m0, omega, t_bc=-1, device="cuda:0", workspace=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the EOFA library has no CPU path")
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        self.dims = tuple(int(d) for d in dims)
        self.Ns = int(Ns)
        self.m0 = float(m0)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        d = (C.c_int * 4)(*self.dims)
        om = self.omega.ctypes.data_as(C.POINTER(C.c_double))
        st = self.lib.eofa_create(C.byref(h), d, self.Ns, self.m0, om, int(t_bc), C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise EofaError(st, "eofa_create failed (see stderr)")
        self.h = h
        self._ws = None
        self._use_ws = workspace
        Lx, Ly, Lz, Lt = self.dims
        self.shape4 = (Lt, Lz, Ly, Lx, 4, 3)
        self.shape5 = (self.Ns,) + self.shape4

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.lib:
                self.lib.eofa_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            msg = self.lib.eofa_last_error(self.h)
            raise EofaError(st, f"{what}: {msg.decode() if msg else ''}")

    def _prep_ws(self, p, nrhs=1):
        if not self._use_ws:
            return
        n = C.c_size_t()
        self._check(self.lib.eofa_workspace_size(self.h, C.byref(p), nrhs, C.byref(n)), "workspace_size")
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = None
            self._ws = self.torch.empty(n.value + 256, dtype=self.torch.uint8, device=self.device)
            addr = self._ws.data_ptr()
            off = (-addr) % 256
            self._check(self.lib.eofa_set_workspace(self.h, C.c_void_p(addr + off), n.value), "set_workspace")

    def _c128(self, t, shape):
        torch = self.torch
        if isinstance(t, np.ndarray):
            t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.complex128))
        t = t.to(device=self.device, dtype=torch.complex128).contiguous()
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
        return t

    def set_gauge(self, U):
        Lx, Ly, Lz, Lt = self.dims
        U = self._c128(U, (Lt, Lz, Ly, Lx, 4, 3, 3))
        self._check(self.lib.eofa_set_gauge(self.h, _ptr(U)), "set_gauge")

    def apply(self, op, x, mp=1.0, mm=1.0, prec=FP64):
        x = self._c128(x, self.shape5)
        out = self.torch.empty_like(x)
        self._prep_ws(params(prec=prec))
        self._check(self.lib.eofa_apply(self.h, OPS[op] if isinstance(op, str) else int(op), float(mp), float(mm),
                                        _ptr(x), _ptr(out), int(prec)), f"apply({op})")
        return out

    def apply_static(self, op, x, mp=1.0, mm=1.0, prec=FP64, out=None):
        """eofa_apply_static: as apply, with no device allocation inside the call (the library's static
        scratch); the caller provides out (allocated here when None).  Waits for the stream."""
        x = self._c128(x, self.shape5)
        if out is None:
            out = self.torch.empty_like(x)
        self._check(self.lib.eofa_apply_static(self.h, OPS[op] if isinstance(op, str) else int(op), float(mp),
                                               float(mm), _ptr(x), _ptr(out), int(prec)), f"apply_static({op})")
        self.torch.cuda.synchronize(self.device)
        return out

    def solve_ht(self, b, mp, mm, p=None):
        p = p or params()
        b = self._c128(b, self.shape5)
        x = self.torch.empty_like(b)
        self._prep_ws(p)
        info = SolveInfo()
        st = self.lib.eofa_solve_ht(self.h, float(mp), float(mm), _ptr(b), _ptr(x), C.byref(p), C.byref(info))
        self._check(st, "solve_ht")
        return x, info.as_dict()

    def solve_ht_batch(self, systems, bs, p=None):
        """systems: list of (m_plus, m_minus); bs: list of 5D sources; returns [(x, info)]."""
        p = p or params()
        n = len(systems)
        bs = [self._c128(b, self.shape5) for b in bs]
        xs = [self.torch.empty_like(b) for b in bs]
        self._prep_ws(p, n)
        mp = (C.c_double * n)(*[float(a[0]) for a in systems])
        mm = (C.c_double * n)(*[float(a[1]) for a in systems])
        pb = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
        px = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        info = (SolveInfo * n)()
        st = self.lib.eofa_solve_ht_batch(self.h, n, mp, mm, pb, px, C.byref(p), info)
        self._check(st, "solve_ht_batch")
        return [(xs[j], info[j].as_dict()) for j in range(n)]

    def chiral_heatbath(self, chir, m3, m4, mo, eta, rel_err=1e-12, lo=0.0, hi=0.0, verify=False, p=None):
        """phi = A^{-1/2} P_c eta for the chiral action A (chir, m3, m4, mo); returns (phi, info)."""
        p = p or params()
        eta = self._c128(eta, self.shape4)
        phi = self.torch.empty_like(eta)
        self._prep_ws(p, HB_BATCH)
        info = HeatbathInfo()
        st = self.lib.eofa_chiral_heatbath(self.h, int(chir), float(m3), float(m4), float(mo), _ptr(eta), _ptr(phi),
                                           float(lo), float(hi), float(rel_err), int(bool(verify)), C.byref(p),
                                           C.byref(info))
        self._check(st, "chiral_heatbath")
        return phi, info.as_dict()

    def heatbath(self, eta, m_lo, m_hi, rel_err=1e-12, verify=False, p=None):
        """phi with weight exp(-phi^dag H^{-1}(m_hi, m_lo) phi); returns (phi, [info_minus, info_plus])."""
        p = p or params()
        eta = self._c128(eta, self.shape4)
        phi = self.torch.empty_like(eta)
        self._prep_ws(p, HB_BATCH)
        info = (HeatbathInfo * 2)()
        st = self.lib.eofa_heatbath(self.h, float(m_lo), float(m_hi), _ptr(eta), _ptr(phi), float(rel_err),
                                    int(bool(verify)), C.byref(p), info)
        self._check(st, "heatbath")
        return phi, [i.as_dict() for i in info]

    def set_workspace(self, buf):
        """Hand the library a caller-owned device buffer (a torch tensor, kept alive here) as its workspace."""
        self._use_ws = False
        self._ws = buf
        addr = buf.data_ptr()
        self._check(self.lib.eofa_set_workspace(self.h, C.c_void_p(addr), buf.numel() * buf.element_size()),
                    "set_workspace")

    def workspace_size(self, p=None, nrhs=1):
        n = C.c_size_t()
        self._check(self.lib.eofa_workspace_size(self.h, C.byref(p or params()), int(nrhs), C.byref(n)),
                    "workspace_size")
        return n.value

    def chiral_action(self, chir, m3, m4, mo, phi, p=None):
        p = p or params()
        phi = self._c128(phi, self.shape4)
        out = self.torch.empty_like(phi)
        self._prep_ws(p)
        S = C.c_double()
        info = SolveInfo()
        st = self.lib.eofa_chiral_action(self.h, int(chir), float(m3), float(m4), float(mo), _ptr(phi), _ptr(out),
                                         C.byref(S), C.byref(p), C.byref(info))
        self._check(st, "chiral_action")
        return Result(out, S.value, [info.as_dict()])

    def chiral_force(self, chir, m3, m4, mo, phi, p=None):
        """Fermion force of one chiral action: (F[mu][t][z][y][x][a] float64 on the device, S, info)."""
        p = p or params()
        phi = self._c128(phi, self.shape4)
        Lx, Ly, Lz, Lt = self.dims
        F = self.torch.empty((4, Lt, Lz, Ly, Lx, 8), dtype=self.torch.float64, device=phi.device)
        self._prep_ws(p)
        S = C.c_double()
        info = SolveInfo()
        st = self.lib.eofa_chiral_force(self.h, int(chir), float(m3), float(m4), float(mo), _ptr(phi), _ptr(F),
                                        C.byref(S), C.byref(p), C.byref(info))
        self._check(st, "chiral_force")
        return F, S.value, info.as_dict()

    def _links(self, U):
        Lx, Ly, Lz, Lt = self.dims
        return self._c128(U, (Lt, Lz, Ly, Lx, 4, 3, 3))

    def gauge_action(self, U, beta):
        """Wilson plaquette action S_g of the canonical links U."""
        U = self._links(U)
        S = C.c_double()
        self._check(self.lib.eofa_gauge_action(self.h, _ptr(U), float(beta), C.byref(S)), "gauge_action")
        return S.value

    def gauge_force(self, U, beta):
        """F[mu][t][z][y][x][a] = dS_g/dw^a (float64 on the device)."""
        U = self._links(U)
        Lx, Ly, Lz, Lt = self.dims
        F = self.torch.empty((4, Lt, Lz, Ly, Lx, 8), dtype=self.torch.float64, device=U.device)
        self._check(self.lib.eofa_gauge_force(self.h, _ptr(U), float(beta), _ptr(F)), "gauge_force")
        return F

    def md_trajectory(self, U, P, actions, beta, tau, steps, metropolis_u=-1.0, p=None, chrono=False, force_tol=0.0):
        """One molecular-dynamics trajectory, in place on U (complex128 [t][z][y][x][mu][3][3]) and P (float64
        [mu][t][z][y][x][8]), both device tensors.  actions: list of (level, chir, m3, m4, mo, phi); steps: total
        steps per level, innermost (gauge) first.  Returns the info dict."""
        torch = self.torch
        Lx, Ly, Lz, Lt = self.dims
        assert isinstance(U, torch.Tensor) and U.dtype == torch.complex128 and U.is_contiguous()
        assert tuple(U.shape) == (Lt, Lz, Ly, Lx, 4, 3, 3) and U.device.type == "cuda"
        assert isinstance(P, torch.Tensor) and P.dtype == torch.float64 and P.is_contiguous()
        assert tuple(P.shape) == (4, Lt, Lz, Ly, Lx, 8) and P.device.type == "cuda"
        p = p or params()
        phis = [self._c128(a[5], self.shape4) for a in actions]
        acts = (MdAction * max(1, len(actions)))()
        for i, (lev, chir, m3, m4, mo, _) in enumerate(actions):
            acts[i] = MdAction(int(chir), float(m3), float(m4), float(mo), int(lev), phis[i].data_ptr())
        steps = list(steps)
        md = MdParams(float(beta), float(tau), len(steps), (C.c_int * 4)(*(steps + [0] * (4 - len(steps)))),
                      float(metropolis_u), int(bool(chrono)), float(force_tol))
        self._prep_ws(p)
        info = MdInfo()
        st = self.lib.eofa_md_trajectory(self.h, _ptr(U), _ptr(P), len(actions), acts, C.byref(md), C.byref(p),
                                         C.byref(info))
        self._check(st, "md_trajectory")
        return info.as_dict()

    def hinv(self, phi, m_lo, m_hi, p=None):
        p = p or params()
        phi = self._c128(phi, self.shape4)
        out = self.torch.empty_like(phi)
        self._prep_ws(p)
        S = C.c_double()
        info = (SolveInfo * 2)()
        st = self.lib.eofa_hinv(self.h, float(m_lo), float(m_hi), _ptr(phi), _ptr(out), C.byref(S), C.byref(p), info)
        self._check(st, "hinv")
        return Result(out, S.value, [i.as_dict() for i in info])

    def chiral_action_batch(self, actions, phis, p=None):
        """actions: list of (chir, m3, m4, mo); phis: list of 4D tensors."""
        p = p or params()
        n = len(actions)
        phis = [self._c128(f, self.shape4) for f in phis]
        outs = [self.torch.empty_like(f) for f in phis]
        self._prep_ws(p, n)
        chir = (C.c_int * n)(*[int(a[0]) for a in actions])
        m3 = (C.c_double * n)(*[float(a[1]) for a in actions])
        m4 = (C.c_double * n)(*[float(a[2]) for a in actions])
        mo = (C.c_double * n)(*[float(a[3]) for a in actions])
        pin = (C.c_void_p * n)(*[f.data_ptr() for f in phis])
        pout = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        S = (C.c_double * n)()
        info = (SolveInfo * n)()
        st = self.lib.eofa_chiral_action_batch(self.h, n, chir, m3, m4, mo, pin, pout, S, C.byref(p), info)
        self._check(st, "chiral_action_batch")
        return [Result(outs[j], S[j], [info[j].as_dict()]) for j in range(n)]

    def dslash_bench(self, nrep=20, prec=FP64):
        ms, b = C.c_double(), C.c_double()
        self._prep_ws(params(prec=prec))
        self._check(self.lib.eofa_dslash_bench(self.h, int(prec), int(nrep), C.byref(ms), C.byref(b)), "dslash_bench")
        return dict(ms=ms.value, bytes=b.value, gbs=b.value / (ms.value * 1e-3) / 1e9)

    def set_schedule(self, sched, prec=FP64):
        """Set the hop schedule (7 ints, as autotune returns them) for storage prec."""
        arr = (C.c_int * 7)(*[int(v) for v in sched])
        self._check(self.lib.eofa_set_schedule(self.h, int(prec), arr), "set_schedule")

    def schedule_candidates(self, prec=FP64):
        """The schedules autotune times for this lattice and storage prec, in its order (lists of 7 ints)."""
        n = C.c_int()
        self._check(self.lib.eofa_schedule_candidates(self.h, int(prec), 0, None, C.byref(n)), "schedule_candidates")
        rows = (C.c_int * (7 * max(n.value, 1)))()
        self._check(self.lib.eofa_schedule_candidates(self.h, int(prec), n.value, rows, C.byref(n)),
                    "schedule_candidates")
        return [list(rows[7 * i:7 * i + 7]) for i in range(n.value)]

    def autotune(self, prec=FP64, nrep=4, cache=None):
        """Pick the hop schedule for this lattice; cache: JSON path keyed by (dims, Ns, prec, arch)."""
        import json
        key = f"{'x'.join(map(str, self.dims))}_Ns{self.Ns}_p{int(prec)}_{self._arch()}"
        sched = (C.c_int * 7)()
        self._prep_ws(params(prec=prec))
        if cache and os.path.exists(cache):
            try:
                with open(cache) as f:
                    entry = json.load(f).get(key)
                if entry and len(entry.get("sched", [])) == 7:
                    sched[:] = entry["sched"]
                    if self.lib.eofa_set_schedule(self.h, int(prec), sched) == OK:
                        return dict(entry, cached=True)
            except (OSError, ValueError):
                pass
        best, base = C.c_double(), C.c_double()
        self._check(self.lib.eofa_autotune(self.h, int(prec), int(nrep), sched, C.byref(best), C.byref(base)),
                    "autotune")
        entry = dict(sched=list(sched), best_ms=best.value, base_ms=base.value)
        if cache:
            try:
                data = {}
                if os.path.exists(cache):
                    with open(cache) as f:
                        data = json.load(f)
                data[key] = entry
                os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
                with open(cache, "w") as f:
                    json.dump(data, f, indent=1, sort_keys=True)
            except (OSError, ValueError):
                pass
        return dict(entry, cached=False)

    def _arch(self):
        try:
            return self.torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        except Exception:
            return "gfx"

    def hinv_batch(self, pairs, phis, p=None):
        """pairs: list of (m_lo, m_hi); phis: list of 4D sources; returns a Result per source."""
        p = p or params()
        n = len(pairs)
        phis = [self._c128(f, self.shape4) for f in phis]
        outs = [self.torch.empty_like(f) for f in phis]
        self._prep_ws(p, 2 * n)
        mlo = (C.c_double * n)(*[float(a[0]) for a in pairs])
        mhi = (C.c_double * n)(*[float(a[1]) for a in pairs])
        pin = (C.c_void_p * n)(*[f.data_ptr() for f in phis])
        pout = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        S = (C.c_double * n)()
        info = (SolveInfo * (2 * n))()
        st = self.lib.eofa_hinv_batch(self.h, n, mlo, mhi, pin, pout, S, C.byref(p), info)
        self._check(st, "hinv_batch")
        return [Result(outs[j], S[j], [info[2 * j].as_dict(), info[2 * j + 1].as_dict()]) for j in range(n)]

    def graph_stats(self):
        n, c = C.c_long(), C.c_int()
        self._check(self.lib.eofa_graph_stats(self.h, C.byref(n), C.byref(c)), "graph_stats")
        return {"replays": n.value, "cached": c.value}

    # ---- learned preconditioner
    def cnn_init(self, seed=0, relu=False):
        self._check(self.lib.eofa_cnn_init(self.h, int(seed), int(bool(relu))), "cnn_init")

    def set_precond(self, params_f32, relu=False):
        w = np.ascontiguousarray(np.asarray(params_f32, dtype=np.float32).reshape(-1))
        self._check(self.lib.eofa_set_precond(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size,
                                              int(bool(relu))), "set_precond")

    def cnn_params(self):
        w = np.empty(CNN_NPARAM, dtype=np.float32)
        self._check(self.lib.eofa_cnn_params(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), "cnn_params")
        return w

    def cnn_apply(self, x5):
        x5 = self._c128(x5, self.shape5)
        out = self.torch.empty_like(x5)
        self._prep_ws(params())
        self._check(self.lib.eofa_cnn_apply(self.h, _ptr(x5), _ptr(out)), "cnn_apply")
        return out

    def cnn_train_step(self, rho5, e5, lr=1e-3, want_grad=False):
        rho5 = self._c128(rho5, self.shape5)
        e5 = self._c128(e5, self.shape5)
        self._prep_ws(params())
        loss = C.c_double()
        g = np.empty(CNN_NPARAM, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        self._check(self.lib.eofa_cnn_train_step(self.h, _ptr(rho5), _ptr(e5), float(lr), C.byref(loss), gp),
                    "cnn_train_step")
        return (loss.value, g) if want_grad else loss.value

    def training_pairs(self, mp, mm, seed, n=8):
        self._prep_ws(params())
        rho = [self.torch.empty(self.shape5, dtype=self.torch.complex128, device=self.device) for _ in range(n)]
        e = [self.torch.empty(self.shape5, dtype=self.torch.complex128, device=self.device) for _ in range(n)]
        pr = (C.c_void_p * n)(*[t.data_ptr() for t in rho])
        pe = (C.c_void_p * n)(*[t.data_ptr() for t in e])
        made = C.c_int()
        self._check(self.lib.eofa_training_pairs(self.h, float(mp), float(mm), int(seed), n, pr, pe, C.byref(made)),
                    "training_pairs")
        return list(zip(rho[:made.value], e[:made.value]))

    def kernel_timing(self, enable=True, reset=False):
        """Per-kernel device time of the FP64 CG iterations: {name: dict(ms, launches, bytes)} for K1..K5."""
        st = KernelStats()
        self._check(self.lib.eofa_kernel_timing(self.h, int(enable), int(reset), C.byref(st)), "kernel_timing")
        return {KERNELS[k]: dict(ms=st.ms[k], launches=st.launches[k], bytes=st.bytes[k]) for k in range(NKERN)}

    def cg_block(self, chir, m3, m4, phi, niter):
        """Source build + even-odd preparation of one chiral action, then exactly niter FP64 CG iterations;
        returns |r_niter| / |r_0| of the normal residual."""
        phi = self._c128(phi, self.shape4)
        self._prep_ws(params())
        rel = C.c_double()
        self._check(self.lib.eofa_cg_block(self.h, int(chir), float(m3), float(m4), _ptr(phi), int(niter),
                                           C.byref(rel)), "cg_block")
        return rel.value
