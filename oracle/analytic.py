"""Closed-form references used to pin the oracle (test infrastructure only).

* equilibrium interface profile phi = tanh(2 r / W)     eq:equilibrium_profile
* Laplace law Delta p = sigma / R                         Sec. 4.3
* Prosperetti's capillary-wave amplitude h(t)/H0          Sec. 4.4, eq:capillary_wave,
  eq:error_function, eq:z (equal kinematic viscosities)
* a circular drop translated by a uniform velocity        Sec. "Effect of parameter
  lambda" (its exact solution after eq:lambda_effect_initial)
"""

import numpy as np
from scipy.special import erfc, wofz


def tanh_profile(r, W):
    return np.tanh(2.0 * np.asarray(r) / W)


def translated_drop(nx, ny, xc, yc, R, W, shift_x):
    """tanh(2 (R - r) / W) about (xc + shift_x, yc), periodic in x."""
    x, y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       indexing="xy")
    dx = x - xc - shift_x
    dx = dx - nx * np.round(dx / nx)
    return np.tanh(2.0 * (R - np.sqrt(dx * dx + (y - yc) ** 2)) / W)


def overshoots(phi):
    """Relative excursions of phi beyond its bulk values, (max phi - 1)/2 and
    (-1 - min phi)/2, zero when inside [-1, 1] (the measures of the lambda tables)."""
    phi = np.asarray(phi)
    return max(0.0, (float(phi.max()) - 1.0) / 2.0), max(0.0, (-1.0 - float(phi.min())) / 2.0)


def laplace_dp(sigma, R):
    return sigma / R


def prosperetti(t, k, nu, sigma, rho_a, rho_b):
    """h(t)/H0 for a planar capillary wave of wave number k (Sec. 4.4).

    beta = rho_a rho_b / (rho_a + rho_b)^2, omega0^2 = sigma k^3 / (rho_a + rho_b);
    z_i are the four roots of the quartic in the paper and Z_i = prod_{j!=i}(z_j - z_i).
    The products e^{z^2 t} erfc(z sqrt t) are evaluated as w(i z sqrt t) (Faddeeva)
    so that large arguments do not overflow.
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    beta = rho_a * rho_b / (rho_a + rho_b) ** 2
    w02 = sigma * k ** 3 / (rho_a + rho_b)
    nk2 = nu * k * k
    coef = [1.0,
            -4.0 * beta * np.sqrt(nk2),
            2.0 * (1.0 - 6.0 * beta) * nk2,
            4.0 * (1.0 - 3.0 * beta) * nk2 ** 1.5,
            (1.0 - 4.0 * beta) * nk2 ** 2 + w02]
    z = np.roots(coef).astype(np.complex128)
    Z = np.array([np.prod([z[j] - z[i] for j in range(4) if j != i]) for i in range(4)])
    first = 4.0 * (1.0 - 4.0 * beta) * nk2 ** 2 / (8.0 * (1.0 - 4.0 * beta) * nk2 ** 2 + w02) \
        * erfc(np.sqrt(nk2 * t))
    tot = np.zeros_like(t, dtype=np.complex128)
    for i in range(4):
        tot += (z[i] / Z[i]) * (w02 / (z[i] ** 2 - nk2)) * np.exp(-nk2 * t) \
            * wofz(1j * z[i] * np.sqrt(t))
    return first + tot.real, np.sqrt(w02)
