"""Pins of the oracle's closed-form references and of its |grad phi| regularisation.

* Prosperetti's capillary-wave amplitude (Sec. 4.4, eq:capillary_wave,
  eq:error_function, eq:z), checked against facts that do not come from its
  own formula: the initial amplitude, the inviscid capillary-wave frequency,
  dimensional consistency (it depends on the densities only through their
  ratio and sigma / (rho_a + rho_b)) and, for a free surface (one density
  negligible), the normal mode of Lamb's viscous dispersion relation.
* the interface height of a column (the capillary wave's amplitude, Sec. 4.4):
  exact on a linear column, second order on a sampled tanh profile.
* the stationarity of the tanh profile (eq:equilibrium_profile) under the FD
  sub-step at the default regularisation eps = 1e-2: the departure from the
  eps -> 0 operator equals the divergence of the closed-form flux
  lambda (sqrt(G^2 + eps^2) - G) n.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
from oracle import diagnostics as D
from oracle import step as S

K_WAVE = 2 * math.pi / 128


@pytest.mark.parametrize("nu,sigma,ra,rb", [
    (0.01, 0.02, 1.0, 1.0),          # equal densities (beta = 1/4)
    (1e-3, 1e-3, 1.0, 1e-3),         # the capillary-wave workload's 1000:1
    (1e-3, 1e-3, 1.0, 0.1),
    (3e-2, 5e-3, 2.0, 0.5),
])
def test_prosperetti_starts_at_the_initial_amplitude(nu, sigma, ra, rb):
    """h(0) = H0: the solution of the initial-value problem starts from the
    imposed perturbation (at rest)."""
    h, _ = A.prosperetti([0.0], K_WAVE, nu, sigma, ra, rb)
    assert abs(h[0] - 1.0) < 1e-10


def test_prosperetti_inviscid_limit_is_the_capillary_wave():
    """nu -> 0: h/H0 -> cos(omega0 t) with the inviscid dispersion relation of
    capillary waves between two fluids, omega0^2 = sigma k^3 / (rho_a + rho_b)."""
    sigma, ra, rb = 1e-3, 1.0, 1e-3
    w0 = math.sqrt(sigma * K_WAVE ** 3 / (ra + rb))
    t = np.linspace(0.0, 3 * 2 * math.pi / w0, 301)
    errs = []
    for nufac in (1e-6, 1e-8, 1e-10):
        h, w = A.prosperetti(t, K_WAVE, nufac * w0 / K_WAVE ** 2, sigma, ra, rb)
        assert abs(w - w0) <= 1e-14 * w0
        errs.append(float(np.abs(h - np.cos(w0 * t)).max()))
    assert errs[2] < 1e-5
    assert errs[0] > errs[1] > errs[2]          # converges as nu -> 0


def test_prosperetti_depends_on_density_ratio_and_sigma_over_density():
    """Scaling both densities and sigma by the same factor leaves the motion
    unchanged (the equations see only rho_b / rho_a and sigma / rho); swapping
    the two fluids leaves it unchanged too (a small-amplitude wave is
    symmetric in which fluid lies below)."""
    t = np.linspace(0.0, 2e4, 401)
    ref, _ = A.prosperetti(t, K_WAVE, 1e-3, 1e-3, 1.0, 0.2)
    for s in (3.0, 0.25):
        h, _ = A.prosperetti(t, K_WAVE, 1e-3, s * 1e-3, s * 1.0, s * 0.2)
        assert np.abs(h - ref).max() < 1e-9
    h, _ = A.prosperetti(t, K_WAVE, 1e-3, 1e-3, 0.2, 1.0)
    assert np.abs(h - ref).max() < 1e-9


def test_prosperetti_free_surface_normal_mode():
    """One density negligible (beta -> 0): a free surface.  At late times the
    amplitude follows the least damped normal mode exp(s t), s a root of Lamb's
    dispersion relation (s + 2 nu k^2)^2 + omega0^2 = 4 nu^2 k^4 sqrt(1 + s/(nu k^2)).
    At omega0 = nu k^2 the root is s = nu k^2 [(sqrt2 - 2) + i (sqrt2 - 1)]
    (checked below); at small nu the decay rate tends to Lamb's 2 nu k^2."""
    sigma, ra, rb = 1e-3, 1.0, 1e-9
    w0 = math.sqrt(sigma * K_WAVE ** 3 / (ra + rb))
    # omega0 = nu k^2
    nu = w0 / K_WAVE ** 2
    a = nu * K_WAVE ** 2
    s = a * complex(math.sqrt(2) - 2, math.sqrt(2) - 1)
    assert abs((s + 2 * a) ** 2 + w0 ** 2 - 4 * a * a * np.sqrt(1 + s / a)) < 1e-12 * a * a
    t = np.linspace(0.0, 30.0 / abs(s.real), 20001)
    h, _ = A.prosperetti(t, K_WAVE, nu, sigma, ra, rb)
    late = t > 10.0 / abs(s.real)
    basis = np.stack([np.exp(s.real * t[late]) * np.cos(s.imag * t[late]),
                      np.exp(s.real * t[late]) * np.sin(s.imag * t[late])], axis=1)
    coef, *_ = np.linalg.lstsq(basis, h[late], rcond=None)
    resid = np.abs(basis @ coef - h[late]).max() / np.abs(h[late]).max()
    assert resid < 1e-4, resid
    # small viscosity: envelope decay rate -> 2 nu k^2 (relative correction ~ sqrt(nu k^2/omega0))
    rates = []
    for nufac in (1e-3, 1e-4):
        nu = nufac * w0 / K_WAVE ** 2
        T = 2 * math.pi / w0
        t = np.linspace(0.0, 400 * T, 400 * 64 + 1)
        h, _ = A.prosperetti(t, K_WAVE, nu, sigma, ra, rb)
        pk = np.nonzero((h[1:-1] > h[:-2]) & (h[1:-1] > h[2:]))[0] + 1
        pk = pk[t[pk] > 20 * T]
        slope = np.polyfit(t[pk], np.log(h[pk]), 1)[0]
        rates.append(-slope / (2 * nu * K_WAVE ** 2))
    assert abs(rates[0] - 1) < 0.03 and abs(rates[1] - 1) < 0.01
    assert abs(rates[1] - 1) < abs(rates[0] - 1)


def test_interface_height_exact_on_a_linear_column():
    y = np.arange(64, dtype=np.float64)
    for y0 in (10.25, 31.5, 40.875):
        col = 0.3 * (y0 - y)
        phi = torch.tensor(np.repeat(col[:, None], 3, axis=1))
        assert abs(D.interface_height(phi, x=1) - y0) < 1e-12
    # no sign change: no interface
    assert math.isnan(D.interface_height(torch.ones(8, 2, dtype=torch.float64)))


def test_interface_height_second_order_on_tanh():
    """The linear interpolation of the zero of a sampled tanh(2 (y0 - y)/W)
    profile is O(h^2) accurate in the node spacing relative to W."""
    errs = []
    for W in (4.0, 8.0, 16.0):
        y = np.arange(256, dtype=np.float64)
        e = 0.0
        for y0 in np.linspace(100.05, 100.95, 19):
            phi = torch.tensor(np.repeat(np.tanh(2 * (y0 - y) / W)[:, None], 2, axis=1))
            e = max(e, abs(D.interface_height(phi, x=0) - y0))
        errs.append(e)
    assert errs[0] < 1e-2
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def _tanh_slab(W, n):
    y = torch.arange(n, dtype=torch.float64)
    r = torch.minimum(y - n / 4, 3 * n / 4 - y)    # two interfaces on a periodic line
    return torch.tanh(2 * r / W)[:, None].expand(n, 8).contiguous()


@pytest.mark.parametrize("lam,M", [(0.005, 0.0), (0.005, 0.02), (0.05, 0.0)])
def test_tanh_stationarity_at_default_eps(lam, M):
    """With eps > 0 the profile flux lambda J_phi no longer vanishes on tanh:
    with the exact gradient G = phi' = 2 (1 - phi^2)/W the flux is
    j = lambda (sqrt(G^2 + eps^2) - G) G / sqrt(G^2 + eps^2), largest where
    G ~ eps (|phi| ~ 0.99 at W = 4).  L(tanh) at eps = 1e-2 departs from its
    eps -> 0 value by the divergence of that flux: between half and 1.1 times
    max |dj/dy| of the closed form (the fourth-order difference of a flux that
    varies over ~W/4 nodes).  The default configuration's drift of the tanh
    profile per step is then at most max |L(tanh; eps -> 0)| (the stencils'
    own error, pinned elsewhere) plus this bound: 7.2e-6 lambda/0.005 per step."""
    W, n, eps = 4.0, 128, 1e-2
    phi = _tanh_slab(W, n)
    base = dict(nx=8, ny=n, W=W, lam=lam, M=M, sigma=0.01)
    Le = S.fd_rhs(phi, oracle.Params(eps=eps, **base))
    L0 = S.fd_rhs(phi, oracle.Params(eps=1e-12, **base))
    r = np.linspace(-30.0, 30.0, 600001)
    G = (2 / W) * (1 - np.tanh(2 * r / W) ** 2)
    mag = np.sqrt(G * G + eps * eps)
    j = lam * (mag - G) * G / mag
    djmax = float(np.abs(np.gradient(j, r)).max())
    d = float((Le - L0).abs().max())
    print(f"lam={lam} M={M}: max|L_eps - L_0| = {d:.3e}, closed-form max|dj/dy| = {djmax:.3e}")
    assert 0.5 * djmax <= d <= 1.1 * djmax
    assert float(Le.abs().max()) <= float(L0.abs().max()) + 1.1 * djmax
    assert abs(djmax / (lam / 0.005) - 7.18e-6) < 0.05e-6
