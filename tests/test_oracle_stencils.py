"""Pins of the oracle's discrete operators.

* isotropic gradient exact on quadratics, isotropic Laplacian exact on cubics
  (eq:dicretized); their Fourier symbols;
* fourth-order difference exact on quartics, symbol i(8 sin k - sin 2k)/6
  (eq:fourOrder_FDM);
* explicit selective filter: on cos(k.x) the output is (1 - a[D(kx)+D(ky)]) cos(k.x)
  with D(k) = d0 + 2 sum d_m cos(mk) (eq:filter, App. B);
* compact filter: its coefficients satisfy the defining conditions, the N=2 and
  N=5 families agree with hand-derived / published closed forms, the FFT line
  solve agrees with a dense circulant solve, and the wall solve keeps the
  mirror symmetry;
* boundary extension: periodic wrap and half-way mirror with parity.
"""

import math

import numpy as np
import pytest
import torch

from oracle import ops, compact
from oracle.lattice import FILTER_D


def _poly_grid(n, fn):
    y, x = torch.meshgrid(torch.arange(n, dtype=torch.float64) - n // 2,
                          torch.arange(n, dtype=torch.float64) - n // 2 + 0.5, indexing="ij")
    return x, y, fn(x, y)


def test_iso_grad_exact_on_quadratics_and_lap_on_cubics():
    x, y, P = _poly_grid(12, lambda x, y: 0.3 + 1.1 * x - 0.7 * y + 0.4 * x * x
                         - 0.25 * x * y + 0.6 * y * y)
    gx, gy = ops.iso_grad(P)
    xi, yi = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert torch.allclose(gx, 1.1 + 0.8 * xi - 0.25 * yi, atol=1e-12)
    assert torch.allclose(gy, -0.7 - 0.25 * xi + 1.2 * yi, atol=1e-12)
    x, y, P = _poly_grid(12, lambda x, y: 0.2 * x ** 3 - 0.1 * x * x * y + 0.3 * y ** 3
                         + 0.5 * x * y + x * x)
    lap = ops.iso_lap(P)
    xi, yi = x[1:-1, 1:-1], y[1:-1, 1:-1]
    ref = (1.2 * xi - 0.2 * yi + 2.0) + (1.8 * yi)
    assert torch.allclose(lap, ref, atol=1e-11)


@pytest.mark.parametrize("k", [(1, 0), (2, 3), (5, 7), (16, 16)])
def test_iso_fourier_symbols(k):
    n = 32
    kx, ky = (2 * math.pi * k[0] / n, 2 * math.pi * k[1] / n)
    y, x = torch.meshgrid(torch.arange(n, dtype=torch.float64),
                          torch.arange(n, dtype=torch.float64), indexing="ij")
    ph = kx * x + ky * y
    c, s = torch.cos(ph), torch.sin(ph)
    gx, gy = ops.iso_grad(ops.ext(c, 1))
    sym_x = (2 / 3) * math.sin(kx) + (1 / 3) * math.sin(kx) * math.cos(ky)
    sym_y = (2 / 3) * math.sin(ky) + (1 / 3) * math.sin(ky) * math.cos(kx)
    assert torch.allclose(gx, -sym_x * s, atol=1e-13)
    assert torch.allclose(gy, -sym_y * s, atol=1e-13)
    lap = ops.iso_lap(ops.ext(c, 1))
    sym_l = (2 / 3) * (2 * math.cos(kx) + 2 * math.cos(ky) - 4) \
        + (1 / 6) * (4 * math.cos(kx) * math.cos(ky) - 4)
    assert torch.allclose(lap, sym_l * c, atol=1e-13)


def test_d4_exact_on_quartics_and_symbol():
    x, y, P = _poly_grid(14, lambda x, y: 0.1 * x ** 4 - 0.2 * x ** 3 + x * y + 0.05 * y ** 4
                         + 0.3 * y ** 3 * x)
    xi, yi = x[2:-2, 2:-2], y[2:-2, 2:-2]
    assert torch.allclose(ops.d4x(P), 0.4 * xi ** 3 - 0.6 * xi ** 2 + yi + 0.3 * yi ** 3,
                          atol=1e-10)
    assert torch.allclose(ops.d4y(P), xi + 0.2 * yi ** 3 + 0.9 * yi ** 2 * xi, atol=1e-10)
    n = 24
    for kk in (1, 3, 7, 12):
        k = 2 * math.pi * kk / n
        y, x = torch.meshgrid(torch.arange(n, dtype=torch.float64),
                              torch.arange(n, dtype=torch.float64), indexing="ij")
        c = torch.cos(k * x)
        d = ops.d4x(ops.ext(c, 2))
        sym = (8 * math.sin(k) - math.sin(2 * k)) / 6
        assert torch.allclose(d, -sym * torch.sin(k * x), atol=1e-13)


@pytest.mark.parametrize("order", [5, 7, 9, 11])
def test_selective_filter_transfer(order):
    d = FILTER_D[order]
    N = len(d) - 1
    n = 32
    a = 0.5
    y, x = torch.meshgrid(torch.arange(n, dtype=torch.float64),
                          torch.arange(n, dtype=torch.float64), indexing="ij")

    def D(k):
        return d[0] + 2 * sum(d[m] * math.cos(m * k) for m in range(1, N + 1))

    for (i, j) in [(0, 0), (1, 2), (4, 9), (16, 0), (16, 16), (11, 5)]:
        kx, ky = 2 * math.pi * i / n, 2 * math.pi * j / n
        c = torch.cos(kx * x + ky * y)
        out = ops.selective_filter(ops.ext(c, N), d, a)
        assert torch.allclose(out, (1 - a * (D(kx) + D(ky))) * c, atol=1e-12)
    # the mean is preserved (D(0) = 0) and the grid-to-grid mode removed (D(pi) = 1, a = 1/2)
    assert abs(D(0.0)) < 1e-11 and abs(D(math.pi) - 1) < 1e-11


def test_ext_periodic_and_mirror():
    X = torch.arange(12, dtype=torch.float64).reshape(3, 4)
    E = ops.ext(X, 2)
    assert torch.equal(E[2:-2, 2:-2], X)
    assert E[0, 0] == X[1, 2]                      # (-2,-2) -> (1, 2) periodic
    E = ops.ext(X, 2, wall_x=True, wall_y=True, odd=True)
    assert E[2, 1] == -X[0, 0]                     # x = -1 mirrors x = 0, flipped
    assert E[2, 0] == -X[0, 1]                     # x = -2 mirrors x = 1
    assert E[1, 1] == X[0, 0]                      # corner: two flips
    E = ops.ext(X, 1, wall_y=True)
    assert torch.equal(E[0, 1:-1], X[0]) and torch.equal(E[-1, 1:-1], X[-1])


# ---------------------------------------------------------------- compact filter

@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.45, 0.49])
def test_compact_conditions(N, alpha):
    a = compact.coefficients(N, alpha)
    assert abs(compact.transfer(np.array([0.0]), N, alpha)[0] - 1) < 1e-13
    assert abs(compact.transfer(np.array([np.pi]), N, alpha)[0]) < 1e-13
    # flatness: T(w) - 1 = O(w^{2N})
    w1, w2 = 0.02, 0.04
    e1 = abs(compact.transfer(np.array([w1]), N, alpha)[0] - 1)
    e2 = abs(compact.transfer(np.array([w2]), N, alpha)[0] - 1)
    if e1 > 1e-15:
        assert math.log(e2 / e1, 2) > 2 * N - 0.5
    assert a.shape == (N + 1,)


def test_compact_closed_forms():
    for alpha in (0.0, 0.25, 0.45):
        # hand-derived N = 2 family
        a = compact.coefficients(2, alpha)
        assert np.allclose(a, [(5 + 6 * alpha) / 8, (1 + 2 * alpha) / 2, (2 * alpha - 1) / 8],
                           atol=1e-15)
        # tenth-order family of Gaitonde & Visbal (AIAA J. 38, 2000)
        a = compact.coefficients(5, alpha)
        ref = [(193 + 126 * alpha) / 256, (105 + 302 * alpha) / 256,
               15 * (-1 + 2 * alpha) / 64, 45 * (1 - 2 * alpha) / 512,
               5 * (-1 + 2 * alpha) / 256, (1 - 2 * alpha) / 512]
        assert np.allclose(a, ref, atol=1e-14)


def test_compact_periodic_fft_equals_dense_circulant_solve():
    n, N, alpha = 24, 5, 0.45
    v = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (3, n)))
    out = compact.lowpass(v, 1, N, alpha, wall=False, odd=False)
    a = compact.coefficients(N, alpha)
    A = np.eye(n)
    B = np.zeros((n, n))
    for i in range(n):
        A[i, (i - 1) % n] += alpha
        A[i, (i + 1) % n] += alpha
        for k in range(N + 1):
            B[i, (i + k) % n] += a[k] / 2
            B[i, (i - k) % n] += a[k] / 2
    ref = np.linalg.solve(A, B @ v.numpy().T).T
    assert np.allclose(out.numpy(), ref, atol=1e-13)


def test_compact_wall_symmetry_and_transfer_in_interior():
    n, N, alpha = 40, 5, 0.45
    # a mirror-symmetric (about the half-way walls) even field stays symmetric
    i = np.arange(n)
    v = np.cos(np.pi * 3 * (i + 0.5) / n)          # even about -1/2 and n-1/2
    out = compact.lowpass(torch.tensor(v)[None, :], 1, N, alpha, wall=True, odd=False)[0].numpy()
    T = compact.transfer(np.array([np.pi * 3 / n]), N, alpha)[0]
    assert np.allclose(out, T * v, atol=1e-13)
    w = np.sin(np.pi * 3 * (i + 0.5) / n)          # odd about the walls
    out = compact.lowpass(torch.tensor(w)[None, :], 1, N, alpha, wall=True, odd=True)[0].numpy()
    assert np.allclose(out, T * w, atol=1e-13)


@pytest.mark.parametrize("wall,odd", [(False, False), (True, False), (True, True)])
@pytest.mark.parametrize("N,alpha", [(5, 0.45), (3, 0.3), (1, -0.2)])
def test_compact_lowpass_is_self_adjoint(wall, odd, N, alpha):
    """The per-direction compact low-pass is a symmetric matrix on periodic
    lines and on lines with half-way mirror ghosts of either parity: the line
    matrix and the right-hand-side stencil are symmetric stencils on the same
    extended line, so they commute.  The library's adjoint of the compact
    filter relies on this (its reverse is the filter itself)."""
    n = 23
    Mx = compact.lowpass(torch.eye(n, dtype=torch.float64), 1, N, alpha, wall=wall, odd=odd)
    M = Mx.numpy()                       # row k = lowpass of the unit vector e_k
    assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
    # and not trivially: the filter is not a multiple of the identity
    assert np.abs(M - np.diag(np.diag(M))).max() > 1e-3


def test_sqrt_is_correctly_rounded():
    """The oracle's sqrt returns the double nearest to the exact square root
    (checked with exact rational arithmetic on random and extreme inputs)."""
    from fractions import Fraction
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(0, 1, 3000), np.exp(rng.normal(0, 30, 3000)),
                         1e-18 + rng.uniform(0, 1e-17, 1000), [0.0, 1.0, 4.0, 1e-300, 2.0]])
    ys = ops.sqrt(torch.tensor(xs)).numpy()
    for x, y in zip(xs, ys):
        X = Fraction(float(x))
        s = Fraction(float(y))
        up = Fraction(float(np.nextafter(y, np.inf)))
        dn = Fraction(float(np.nextafter(y, -np.inf))) if y > 0 else -s
        assert ((s + dn) / 2) ** 2 <= X <= ((s + up) / 2) ** 2, x
    # differentiable: d sqrt(x)/dx = 1/(2 sqrt x)
    t = torch.tensor([0.25, 4.0], dtype=torch.float64, requires_grad=True)
    ops.sqrt(t).sum().backward()
    assert torch.allclose(t.grad, torch.tensor([1.0, 0.25], dtype=torch.float64))
