"""Compact (tridiagonal) selective filter -- the variant the paper names only.

The abstract and the conclusions speak of a "high-order compact selective
filter"; the filter the paper actually defines (eq:filter, App. B) is explicit.
This module defines the compact variant from first principles:

    per line:  alpha chi^_{i-1} + chi^_i + alpha chi^_{i+1}
                   = sum_{n=0..N} (a_n / 2) (chi_{i+n} + chi_{i-n})

whose transfer function is T(w) = sum_n a_n cos(n w) / (1 + 2 alpha cos w).
The N+1 coefficients a_n solve T(0) = 1, T(pi) = 0 and the vanishing of the
w^2 .. w^{2(N-1)} Taylor terms of T(w) - 1, i.e.
    sum_n a_n = 1 + 2 alpha,  sum_n (-1)^n a_n = 0,
    sum_n n^{2k} a_n = 2 alpha   (k = 1 .. N-1).
The filtered field keeps the paper's intensity a and the unsplit form of
eq:filter with the high-pass part (chi - chi^) in place of sum_j d_j chi:
    chi~ = chi - a [ (chi - F_x chi) + (chi - F_y chi) ].

Periodic lines: the line system is circulant, so chi^ is computed exactly in
Fourier space, chi^ = IFFT(T(w_k) FFT(chi)).  Walled lines: the ghost rule of
the other stencils (half-way mirror, sign kept for p, flipped for u) applied
to both chi and chi^, solved densely.
"""

import numpy as np
import torch


def coefficients(N, alpha):
    """a_0..a_N from the conditions in the module docstring (a small linear solve)."""
    A = np.zeros((N + 1, N + 1))
    b = np.zeros(N + 1)
    A[0, :] = 1.0
    b[0] = 1.0 + 2.0 * alpha
    for k in range(1, N):
        for n in range(N + 1):
            A[k, n] = float(n) ** (2 * k)
        b[k] = 2.0 * alpha
    for n in range(N + 1):
        A[N, n] = (-1.0) ** n
    b[N] = 0.0
    return np.linalg.solve(A, b)


def transfer(w, N, alpha):
    a = coefficients(N, alpha)
    num = sum(a[n] * np.cos(n * w) for n in range(N + 1))
    return num / (1.0 + 2.0 * alpha * np.cos(w))


def _lowpass_periodic(X, dim, N, alpha):
    n = X.shape[dim]
    w = 2.0 * np.pi * np.fft.fftfreq(n)
    T = torch.tensor(transfer(w, N, alpha), dtype=torch.float64)
    shape = [1] * X.dim()
    shape[dim] = n
    Xh = torch.fft.fft(X, dim=dim) * T.reshape(shape)
    return torch.fft.ifft(Xh, dim=dim).real


def _lowpass_wall(X, dim, N, alpha, odd):
    n = X.shape[dim]
    a = coefficients(N, alpha)
    sgn = -1.0 if odd else 1.0
    # right-hand side with mirrored ghosts
    Xt = X.movedim(dim, -1)
    idx, sg = [], []
    for i in range(-N, n + N):
        if i < 0:
            idx.append(-1 - i)
            sg.append(sgn)
        elif i >= n:
            idx.append(2 * n - 1 - i)
            sg.append(sgn)
        else:
            idx.append(i)
            sg.append(1.0)
    E = Xt[..., idx] * torch.tensor(sg, dtype=torch.float64)
    rhs = 0
    for k in range(N + 1):
        lo = E[..., N - k:N - k + n]
        hi = E[..., N + k:N + k + n]
        rhs = rhs + (a[k] / 2.0) * (lo + hi)
    A = np.eye(n)
    for i in range(n - 1):
        A[i, i + 1] = alpha
        A[i + 1, i] = alpha
    A[0, 0] += sgn * alpha
    A[n - 1, n - 1] += sgn * alpha
    At = torch.tensor(A, dtype=torch.float64)
    sol = torch.linalg.solve(At, rhs.reshape(-1, n).T).T.reshape(rhs.shape)
    return sol.movedim(-1, dim)


def lowpass(X, dim, N, alpha, wall, odd):
    if wall:
        return _lowpass_wall(X, dim, N, alpha, odd)
    return _lowpass_periodic(X, dim, N, alpha)


def filter2d(X, N, alpha, a, wall_x, wall_y, odd):
    """chi~ = chi - a[(chi - F_x chi) + (chi - F_y chi)] on a (ny, nx) field."""
    Fx = lowpass(X, 1, N, alpha, wall_x, odd)
    Fy = lowpass(X, 0, N, alpha, wall_y, odd)
    return X - a * ((X - Fx) + (X - Fy))
