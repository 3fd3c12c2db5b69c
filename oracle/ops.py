"""Discrete operators on extended (ghost-padded) 2-D fields.

Arrays are ``torch.float64`` with shape ``(ny, nx)``, index ``[y, x]``.
A field "with halo h" has shape ``(ny + 2h, nx + 2h)``; stencil functions take
such an array and return the result on the halo shrunk by the stencil radius
("valid" evaluation), so that every value is computed from ghost-extended
inputs only.

Boundary rules (the paper names only periodic and no-slip boundaries, Sec. 4.4
and Sec. 4.5; the ghost rule is a reading): along a periodic axis ghosts wrap;
along a walled axis the wall sits half-way between the last node and its ghost
(nodes 0..n-1, walls at -1/2 and n-1/2) and the ghost takes the value at the
mirror node, with the sign flipped for velocity components (no-slip) and kept
for phi, mu and p.

Evaluation order: every sum is accumulated left to right in the order written,
zero terms skipped; divisions by c_s^2 = 1/3 are multiplications by 3.
"""

import numpy as np
import torch

from .lattice import C, W

CS2_INV = 3.0  # 1 / c_s^2, exact


class _SqrtCR(torch.autograd.Function):
    """Correctly rounded square root (IEEE 754), differentiable.

    torch's CPU float64 sqrt is off by one ulp on about 1 % of inputs; numpy's
    (the hardware instruction) is correctly rounded, which is what the
    mathematics of |grad phi| asks for."""

    @staticmethod
    def forward(ctx, x):
        y = torch.from_numpy(np.sqrt(x.detach().cpu().numpy()))
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, gy):
        (y,) = ctx.saved_tensors
        return gy / (2 * y)


def sqrt(x):
    return _SqrtCR.apply(x)


def _axis_map(n, h, wall):
    idx, sgn = [], []
    for i in range(-h, n + h):
        if not wall:
            idx.append(i % n)
            sgn.append(1.0)
        elif i < 0:
            idx.append(-1 - i)
            sgn.append(-1.0)
        elif i >= n:
            idx.append(2 * n - 1 - i)
            sgn.append(-1.0)
        else:
            idx.append(i)
            sgn.append(1.0)
    return torch.tensor(idx), torch.tensor(sgn, dtype=torch.float64)


def ext(X, h, wall_x=False, wall_y=False, odd=False):
    """Pad a (ny, nx) field with h ghost layers (periodic wrap or half-way mirror).

    ``odd`` flips the sign of mirrored ghosts (velocity components at a no-slip
    wall).  Requires h <= n along a walled axis.
    """
    ny, nx = X.shape
    iy, sy = _axis_map(ny, h, wall_y)
    ix, sx = _axis_map(nx, h, wall_x)
    Y = X[iy][:, ix]
    if odd:
        Y = Y * (sy[:, None] * sx[None, :])
    return Y


def crop(X, h_from, h_to):
    d = h_from - h_to
    if d == 0:
        return X
    return X[d:X.shape[0] - d, d:X.shape[1] - d]


def S(P, r, dx, dy):
    """P(x + dx, y + dy) on the region of P shrunk by r on every side."""
    ny, nx = P.shape
    return P[r + dy:ny - r + dy, r + dx:nx - r + dx]


def iso_grad(P):
    """Isotropic gradient, eq:dicretized (first line): sum_{i!=0} w_i c_i P(x+c_i) / c_s^2.

    Shrinks the halo by 1.  Returns (d/dx, d/dy).
    """
    gx = 0
    gy = 0
    for i in range(1, 9):
        cx, cy = C[i]
        t = S(P, 1, cx, cy)
        if cx != 0:
            gx = gx + (W[i] * cx) * t
        if cy != 0:
            gy = gy + (W[i] * cy) * t
    return gx * CS2_INV, gy * CS2_INV


def iso_lap(P):
    """Isotropic Laplacian, eq:dicretized (second line):
    sum_{i!=0} 2 w_i (P(x+c_i) - P(x)) / c_s^2.  Shrinks the halo by 1."""
    P0 = S(P, 1, 0, 0)
    acc = 0
    for i in range(1, 9):
        cx, cy = C[i]
        acc = acc + (2 * W[i]) * (S(P, 1, cx, cy) - P0)
    return acc * CS2_INV


def d4x(P):
    """Fourth-order central first derivative along x, eq:fourOrder_FDM
    (read as [P(x-2) - 8P(x-1) + 8P(x+1) - P(x+2)] / 12).  Shrinks the halo by 2."""
    return (((S(P, 2, -2, 0) - 8 * S(P, 2, -1, 0)) + 8 * S(P, 2, 1, 0)) - S(P, 2, 2, 0)) / 12


def d4y(P):
    """Fourth-order central first derivative along y (same reading as d4x)."""
    return (((S(P, 2, 0, -2) - 8 * S(P, 2, 0, -1)) + 8 * S(P, 2, 0, 1)) - S(P, 2, 0, 2)) / 12


def selective_filter(P, d, a):
    """Explicit centred selective filter, eq:filter with d_{-m} = d_m (App. B).

    chi <- chi - a * [ sum_{j=-N..N} d_|j| chi(x+j, y) + sum_j d_|j| chi(x, y+j) ]
    applied unsplit (both directions read the unfiltered input).  P has halo
    >= N = len(d)-1; the result has halo shrunk by N.
    """
    N = len(d) - 1
    sx = 0
    sy = 0
    for j in range(-N, N + 1):
        sx = sx + d[abs(j)] * S(P, N, j, 0)
    for j in range(-N, N + 1):
        sy = sy + d[abs(j)] * S(P, N, 0, j)
    return S(P, N, 0, 0) - a * (sx + sy)
