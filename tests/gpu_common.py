"""Shared helpers of the GPU tests: build the seeded case, run the HIP path, compare with the oracle."""
import numpy as np

from paper_1710_09621_amd import inputs as IN

M0 = 1.3


def case(dims, Ns, eps=0.5, seed=7, tbc=-1):
    U = IN.gauge_links(dims, eps, seed)
    om = IN.optimal_omega(Ns)
    return U, om


def ctx_and_oracle(dims, Ns, eps=0.5, seed=7, tbc=-1):
    from oracle import oracle as O
    from paper_1710_09621_amd import eofa as E
    U, om = case(dims, Ns, eps, seed, tbc)
    ctx = E.Context(dims, Ns, M0, om, t_bc=tbc)
    ctx.set_gauge(U)
    lat = O.Lattice(dims, U, m0=M0, omega=om, tbc=tbc)
    return ctx, lat


def rand5(lat, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(lat.shape5) + 1j * rng.standard_normal(lat.shape5)


def relerr(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
