"""Plain CPU reference of the learned preconditioner network (PyTorch CPU ops).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.  The network is not part of
the paper's method; this module is the plain definition of the map the HIP kernels implement,
written independently of them.

Fields are canonical 5D complex128 arrays [Ns][Lt][Lz][Ly][Lx][4][3].  The network acts on the odd
sites ((x+y+z+t) odd) laid out on the checkerboard-compressed lattice (xh = x // 2, y, z, t) with
periodic wrap, one s-slice at a time, with channels c = 2 (3 spin + colour) + (0 re | 1 im), 24 of
them live, padded to 32.  Layer l computes
    Y[n] = b[n] + sum over (dt, dz, dy, dx) in {-1, 0, 1}^4 of sum_k X(site + d)[k] W[tap][n][k],
    tap = 27 (dt+1) + 9 (dz+1) + 3 (dy+1) + (dx+1),
with channel counts 24 -> 32 -> 32 -> 32 -> 24.  The flat parameter vector holds, per layer, the
weights [81][32][32] and then 32 biases.  ``bf16=True`` rounds the network input, the weights and
the hidden activations to bfloat16, as the kernels store them; arithmetic is in ``dtype``.
"""
from __future__ import annotations

import numpy as np
import torch

LAYERS = 4
CIN = (24, 32, 32, 32)
COUT = (32, 32, 32, 24)
WSZ = 81 * 32 * 32
LSZ = WSZ + 32
NPARAM = LAYERS * LSZ


def tap_index(dt, dz, dy, dx):
    return 27 * (dt + 1) + 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)


def _odd_coords(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, xh = np.indices((Lt, Lz, Ly, Lx // 2))
    x = 2 * xh + ((y + z + t + 1) & 1)
    return t, z, y, x


def odd_rows(psi, dims):
    """canonical 5D complex -> float64 array [Ns][Lt][Lz][Ly][Lx/2][24] of the odd sites"""
    t, z, y, x = _odd_coords(dims)
    v = np.asarray(psi)[:, t, z, y, x]
    v = v.reshape(v.shape[:5] + (12,))
    out = np.empty(v.shape[:-1] + (24,))
    out[..., 0::2] = v.real
    out[..., 1::2] = v.imag
    return out


def rows_to_canonical(rows, dims):
    """inverse of odd_rows (first 24 channels); even sites are zero"""
    Lx, Ly, Lz, Lt = dims
    Ns = rows.shape[0]
    out = np.zeros((Ns, Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)
    t, z, y, x = _odd_coords(dims)
    c = (rows[..., 0:24:2] + 1j * rows[..., 1:24:2]).reshape(rows.shape[:5] + (4, 3))
    out[:, t, z, y, x] = c
    return out


def _bf(x, on):
    return x.to(torch.bfloat16).to(x.dtype) if on else x


def layer_views(p):
    """(W [81][32][32], b [32]) views of a flat parameter tensor, per layer"""
    return [(p[l * LSZ: l * LSZ + WSZ].view(81, 32, 32), p[l * LSZ + WSZ: (l + 1) * LSZ]) for l in range(LAYERS)]


def conv(x, W, b):
    """one layer on x: [Ns][Lt][Lz][Ly][Lx/2][32]"""
    y = torch.zeros(x.shape[:-1] + (32,), dtype=x.dtype)
    for dt in (-1, 0, 1):
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    xs = torch.roll(x, shifts=(-dt, -dz, -dy, -dx), dims=(1, 2, 3, 4))  # xs[i] = x[i + d]
                    y = y + xs @ W[tap_index(dt, dz, dy, dx)].T
    return y + b


def network(x24, p, relu=False, bf16=True):
    """x24: [Ns][Lt][Lz][Ly][Lx/2][24] tensor -> output [..][32] (channels 24..31 of the last layer are 0)"""
    x = torch.zeros(x24.shape[:-1] + (32,), dtype=p.dtype)
    x[..., :24] = x24
    x = _bf(x, bf16)
    for l, (W, b) in enumerate(layer_views(p)):
        x = conv(x, _bf(W, bf16), b)
        if l < LAYERS - 1:
            if relu:
                x = torch.relu(x)
            x = _bf(x, bf16)
    return x


def apply(psi, dims, params, relu=False, bf16=True, dtype=torch.float32):
    """|psi_o| N(psi_o / |psi_o|) on the odd sites, canonical 5D in and out"""
    r = odd_rows(psi, dims)
    nrm = np.sqrt(np.sum(r * r))
    p = torch.as_tensor(np.asarray(params), dtype=dtype)
    y = network(torch.as_tensor(r / nrm, dtype=dtype), p, relu, bf16)
    return rows_to_canonical(nrm * y[..., :24].double().numpy(), dims)


def loss_and_grad(rho, e, dims, params, relu=False, bf16=False, dtype=torch.float32):
    """Training loss of one pair and its gradient.

    Input rho / |rho|, target e / |rho| (odd sites), L = |N - T|^2 / |T|^2.  Returns (L, g) with
    g = dL/dparam * |T|^2 / 2 = d(|N - T|^2 / 2)/dparam, and zeros for the padding channels.
    """
    r = odd_rows(rho, dims)
    t = odd_rows(e, dims)
    nrm = np.sqrt(np.sum(r * r))
    p = torch.tensor(np.asarray(params), dtype=dtype, requires_grad=True)
    T = torch.zeros(r.shape[:-1] + (32,), dtype=dtype)
    T[..., :24] = torch.as_tensor(t / nrm, dtype=dtype)
    y = network(torch.as_tensor(r / nrm, dtype=dtype), p, relu, bf16)
    half_sq = 0.5 * torch.sum((y - T) ** 2)
    half_sq.backward()
    g = p.grad.detach().numpy().copy()
    for l in range(LAYERS):
        Wg = g[l * LSZ: l * LSZ + WSZ].reshape(81, 32, 32)
        Wg[:, COUT[l]:, :] = 0
        Wg[:, :, CIN[l]:] = 0
        g[l * LSZ + WSZ + COUT[l]: (l + 1) * LSZ] = 0
    return 2.0 * half_sq.item() / torch.sum(T * T).item(), g


def layer_terms(rho, e, dims, params, bf16=True, dtype=torch.float32):
    """Per-layer operands of the weight gradient of one training pair (input rho / |rho|, target e / |rho|,
    linear network): X[l] the layer inputs as the convolution reads them ([Ns][Lt][Lz][Ly][Lx/2][32]) and
    dY[l] = d(|N - T|^2 / 2)/d(output of layer l).  The weight gradient of layer l is
    sum over rows of dY[l][row][n] X[l][row + d][k] at tap d (see conv), its bias gradient sum dY[l][row][n]."""
    r = odd_rows(rho, dims)
    t = odd_rows(e, dims)
    nrm = np.sqrt(np.sum(r * r))
    p = torch.as_tensor(np.asarray(params), dtype=dtype)
    T = torch.zeros(r.shape[:-1] + (32,), dtype=dtype)
    T[..., :24] = torch.as_tensor(t / nrm, dtype=dtype)
    x = torch.zeros(r.shape[:-1] + (32,), dtype=dtype)
    x[..., :24] = torch.as_tensor(r / nrm, dtype=dtype)
    x = _bf(x, bf16)
    x.requires_grad_(True)
    X, Y = [], []
    for l, (W, b) in enumerate(layer_views(p)):
        X.append(x)
        y = conv(x, _bf(W, bf16), b)
        Y.append(y)
        x = _bf(y, bf16) if l < LAYERS - 1 else y
    half_sq = 0.5 * torch.sum((x - T) ** 2)
    dY = torch.autograd.grad(half_sq, Y)
    return [v.detach() for v in X], [v.detach() for v in dY]
