"""Pins of the CPU reference network (test infrastructure) against closed forms and finite differences."""
import numpy as np
import torch

from oracle import cnn_ref as R
from paper_1710_09621_amd import inputs as IN


def _field(dims, Ns, seed):
    rng = np.random.default_rng(seed)
    shape = (Ns,) + tuple(reversed(dims)) + (4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _odd_mask(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    return ((x + y + z + t) & 1).astype(bool)


def _identity_params(shift_layer=None, tap=40):
    p = np.zeros(R.NPARAM)
    for l in range(R.LAYERS):
        W = p[l * R.LSZ: l * R.LSZ + R.WSZ].reshape(81, 32, 32)
        W[tap if l == shift_layer else 40, np.arange(24), np.arange(24)] = 1.0
    return p


def test_identity_network_is_identity_on_odd_sites():
    dims, Ns = (4, 2, 2, 2), 8
    psi = _field(dims, Ns, 1)
    out = R.apply(psi, dims, _identity_params(), bf16=False, dtype=torch.float64)
    odd = _odd_mask(dims)
    assert np.abs(out[:, odd] - psi[:, odd]).max() < 1e-13
    assert np.all(out[:, ~odd] == 0)


def test_single_tap_is_a_shift_on_the_compressed_lattice():
    """W = 1 on the tap of d = (dt, dz, dy, dx) maps out(xh, y, z, t) = in(xh+dx, y+dy, z+dz, t+dt) (periodic)."""
    dims, Ns = (6, 4, 2, 2), 2
    Lx, Ly, Lz, Lt = dims
    psi = _field(dims, Ns, 2)
    for d in [(0, 0, 0, 1), (0, 0, -1, 0), (1, 0, 0, 0), (0, 1, 0, -1)]:
        dt, dz, dy, dx = d
        out = R.apply(psi, dims, _identity_params(shift_layer=2, tap=R.tap_index(dt, dz, dy, dx)), bf16=False,
                      dtype=torch.float64)
        for t in range(Lt):
            for z in range(Lz):
                for y in range(Ly):
                    for xh in range(Lx // 2):
                        x = 2 * xh + ((y + z + t + 1) & 1)
                        t2, z2, y2 = (t + dt) % Lt, (z + dz) % Lz, (y + dy) % Ly
                        x2 = 2 * ((xh + dx) % (Lx // 2)) + ((y2 + z2 + t2 + 1) & 1)
                        assert np.abs(out[:, t, z, y, x] - psi[:, t2, z2, y2, x2]).max() < 1e-13


def test_linear_network_is_linear_and_homogeneous():
    """Without biases and activations, |r| N(r / |r|) is linear in r."""
    dims, Ns = (4, 2, 2, 2), 8
    p = IN.cnn_params(3).astype(np.float64)
    for l in range(R.LAYERS):
        p[l * R.LSZ + R.WSZ: (l + 1) * R.LSZ] = 0
    a, b = _field(dims, Ns, 4), _field(dims, Ns, 5)
    f = lambda v: R.apply(v, dims, p, bf16=False, dtype=torch.float64)
    lhs = f(2.0 * a - 0.5 * b)
    rhs = 2.0 * f(a) - 0.5 * f(b)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_bias_reaches_output_through_all_layers():
    """With zero weights the output is the last layer's bias times |r| on every odd site."""
    dims, Ns = (4, 2, 2, 2), 2
    p = np.zeros(R.NPARAM)
    bias = np.arange(1, 25) / 10.0
    p[3 * R.LSZ + R.WSZ: 3 * R.LSZ + R.WSZ + 24] = bias
    psi = _field(dims, Ns, 6)
    out = R.apply(psi, dims, p, bf16=False, dtype=torch.float64)
    nrm = np.sqrt(np.sum(np.abs(psi[:, _odd_mask(dims)]) ** 2))
    want = (bias[0::2] + 1j * bias[1::2]).reshape(4, 3) * nrm
    assert np.abs(out[:, _odd_mask(dims)] - want).max() < 1e-12 * nrm


def test_gradient_matches_central_differences():
    dims, Ns = (4, 2, 2, 2), 8
    p = IN.cnn_params(7).astype(np.float64)
    rho, e = _field(dims, Ns, 8), _field(dims, Ns, 9)
    for relu in (False, True):
        L0, g = R.loss_and_grad(rho, e, dims, p, relu=relu, dtype=torch.float64)
        t = R.odd_rows(e, dims) / np.sqrt(np.sum(R.odd_rows(rho, dims) ** 2))
        t2 = np.sum(t * t)
        rng = np.random.default_rng(10)
        for l in range(R.LAYERS):
            idx = [l * R.LSZ + tap * 1024 + n * 32 + k for tap, n, k in
                   zip(rng.integers(0, 81, 4), rng.integers(0, R.COUT[l], 4), rng.integers(0, R.CIN[l], 4))]
            idx.append(l * R.LSZ + R.WSZ + int(rng.integers(0, R.COUT[l])))
            for i in idx:
                h = 1e-6
                pp, pm = p.copy(), p.copy()
                pp[i] += h
                pm[i] -= h
                Lp, _ = R.loss_and_grad(rho, e, dims, pp, relu=relu, dtype=torch.float64)
                Lm, _ = R.loss_and_grad(rho, e, dims, pm, relu=relu, dtype=torch.float64)
                fd = (Lp - Lm) / (2 * h) * t2 / 2
                assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (relu, l, i, fd, g[i])
    assert L0 > 0
