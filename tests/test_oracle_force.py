"""Pins of the oracle's EOFA fermion force (oracle/force.py): central finite differences of the oracle's
own chiral action S under U_mu(x) -> exp(i h T^a) U_mu(x), on links in the bulk and across the
antiperiodic t boundary, for both chiralities; and the forces of one splitting's actions add up."""
import numpy as np
import pytest
from scipy.linalg import expm

DIMS, NS = (2, 2, 2, 4), 4


@pytest.fixture(scope="module")
def setup(oracle_lib):
    from oracle import oracle as O
    from paper_1710_09621_amd import inputs as IN
    U = IN.gauge_links(DIMS, 0.6, 21)
    om = IN.optimal_omega(NS)
    lat = O.Lattice(DIMS, U, m0=1.3, omega=om, tbc=-1)
    phi = IN.gaussian_spinor(DIMS[::-1], 5)
    return O, IN, U, om, lat, phi


def _S(O, U, om, chir, m3, m4, mo, phi):
    lat = O.Lattice(DIMS, U, m0=1.3, omega=om, tbc=-1)
    return lat.chiral_action(chir, m3, m4, mo, phi, tol=1e-14)[1]


# (mu, t, z, y, x, a): bulk links in every direction, a t link across the boundary (t = Lt - 1), all 8 generators
SAMPLES = [(0, 1, 0, 1, 0, 0), (1, 2, 1, 0, 1, 1), (2, 0, 1, 1, 0, 2), (3, 1, 0, 0, 1, 3), (3, 3, 1, 0, 0, 4),
           (3, 3, 0, 1, 1, 7), (0, 3, 1, 1, 1, 5), (2, 2, 0, 0, 0, 6)]


@pytest.mark.parametrize("chir,m3,m4,mo", [(-1, 0.05, 0.05, 0.3), (+1, 0.05, 0.3, 0.6), (-1, 0.4, 0.1, 1.0)])
def test_force_is_the_derivative_of_the_action(setup, chir, m3, m4, mo):
    from oracle import force as OF
    O, IN, U, om, lat, phi = setup
    F = OF.force(lat, chir, m3, m4, mo, phi, tol=1e-14)
    scale = np.abs(F).max()
    assert scale > 1e-3
    h = 1e-4
    for mu, t, z, y, x, a in SAMPLES:
        Up, Um = U.copy(), U.copy()
        Up[t, z, y, x, mu] = expm(1j * h * OF.T[a]) @ U[t, z, y, x, mu]
        Um[t, z, y, x, mu] = expm(-1j * h * OF.T[a]) @ U[t, z, y, x, mu]
        fd = (_S(O, Up, om, chir, m3, m4, mo, phi) - _S(O, Um, om, chir, m3, m4, mo, phi)) / (2 * h)
        assert abs(fd - F[mu, t, z, y, x, a]) < 1e-6 * scale, (mu, t, z, y, x, a, fd, F[mu, t, z, y, x, a])


def test_generators(setup):
    from oracle import force as OF
    T = OF.T
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-14
