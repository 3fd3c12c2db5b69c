"""Pins of the oracle's equilibria, sources and collision against closed forms.

* moments of f^eq that the CH recovery needs (sum = phi, first = phi u,
  second = eta mu c_s^2 I + phi u u) -- eq:feq_CH with Sec. 3.1's mobility relation;
* M g^eq against the moment vector of App. A (eq:mg0: p/c_s^2, u_x, u_y) and the
  standard second-order entries;
* M G against the structure of App. A's source vector (eq:mG1), with the reading
  b = F/rho - grad p; M F_i (eq:Fi) = (0,0,0, phi a_x, -phi a_x, phi a_y, -phi a_y, 0, 0);
* the MRT collision reduces to BGK with the same forcing when all s_i are equal
  (Sec. 3.1, text after eq:CH_Sf);
* a uniform state at rest is a fixed point of the whole step.
"""

import numpy as np
import torch

import oracle
from oracle import lattice as L
from oracle import step as S


def _rand(shape, seed, lo=-1.0, hi=1.0):
    g = torch.Generator().manual_seed(seed)
    return lo + (hi - lo) * torch.rand(shape, generator=g, dtype=torch.float64)


def _prm(**kw):
    base = dict(nx=8, ny=8, sigma=0.01, M=0.02, tau_f=0.8)
    base.update(kw)
    return oracle.Params(**base)


def test_feq_moments():
    prm = _prm()
    phi, mu, ux, uy = (_rand((5, 7), s) for s in range(4))
    ux = 0.1 * ux
    uy = 0.1 * uy
    f = torch.stack(S.f_eq(phi, mu, ux, uy, prm))
    c = torch.tensor(L.C, dtype=torch.float64)
    assert torch.allclose(f.sum(0), phi, atol=1e-15, rtol=0)
    assert torch.allclose((f * c[:, 0, None, None]).sum(0), phi * ux, atol=1e-15, rtol=0)
    assert torch.allclose((f * c[:, 1, None, None]).sum(0), phi * uy, atol=1e-15, rtol=0)
    eta = prm.eta
    Pxx = (f * (c[:, 0] ** 2)[:, None, None]).sum(0)
    Pxy = (f * (c[:, 0] * c[:, 1])[:, None, None]).sum(0)
    Pyy = (f * (c[:, 1] ** 2)[:, None, None]).sum(0)
    assert torch.allclose(Pxx, eta * mu / 3 + phi * ux * ux, atol=1e-15, rtol=0)
    assert torch.allclose(Pyy, eta * mu / 3 + phi * uy * uy, atol=1e-15, rtol=0)
    assert torch.allclose(Pxy, phi * ux * uy, atol=1e-15, rtol=0)
    # mobility relation eq:mobility: M = eta c_s^2 (tau_f - 1/2)
    assert abs(eta / 3 * (prm.tau_f - 0.5) - prm.M) < 1e-16


def test_geq_moment_vector_app_a():
    p, ux, uy = (_rand((6, 5), s) for s in (10, 11, 12))
    ux = 0.1 * ux
    uy = 0.1 * uy
    m = S.m_apply(S.g_eq(p, ux, uy))
    usq = ux * ux + uy * uy
    ref = [3 * p, -6 * p + 3 * usq, 3 * p - 3 * usq, ux, -ux, uy, -uy, ux * ux - uy * uy, ux * uy]
    for k in range(9):
        assert torch.allclose(m[k], ref[k], atol=2e-15, rtol=0), k


def test_source_moment_vectors():
    Fx, Fy, bx, by, ux, uy = (_rand((4, 6), s) for s in range(20, 26))
    rho = _rand((4, 6), 26, 0.001, 1.0)
    m = S.m_apply(S.src_g(Fx, Fy, rho, ux, uy, bx, by))
    bu = bx * ux + by * uy
    ref = [0 * bu, 6 * bu, -6 * bu, Fx / rho, -Fx / rho, Fy / rho, -Fy / rho,
           2 * (bx * ux - by * uy), bx * uy + by * ux]
    for k in range(9):
        assert torch.allclose(m[k], ref[k], atol=5e-13, rtol=1e-13), k
    phi, ax, ay = (_rand((4, 6), s) for s in range(30, 33))
    m = S.m_apply(S.src_f(phi, ax, ay))
    z = 0 * phi
    ref = [z, z, z, phi * ax, -phi * ax, phi * ay, -phi * ay, z, z]
    for k in range(9):
        assert torch.allclose(m[k], ref[k], atol=2e-15, rtol=0), k


def test_mrt_reduces_to_bgk_when_rates_equal():
    f = [_rand((3, 4), 40 + i) for i in range(9)]
    feq = [_rand((3, 4), 50 + i) for i in range(9)]
    F = [_rand((3, 4), 60 + i) for i in range(9)]
    tau = 0.73
    out = S.mrt_collide(f, feq, F, [1.0 / tau] * 9)
    for i in range(9):
        ref = f[i] - (f[i] - feq[i]) / tau + (1 - 1 / (2 * tau)) * F[i]
        assert torch.allclose(out[i], ref, atol=1e-14, rtol=0)


def test_mrt_against_dense_matrices():
    """Brute force: Lambda = inv(M) S M as a dense 9x9 matrix (numpy.linalg.inv)."""
    f = np.random.default_rng(1).uniform(-1, 1, 9)
    feq = np.random.default_rng(2).uniform(-1, 1, 9)
    F = np.random.default_rng(3).uniform(-1, 1, 9)
    s = np.array([1.0, 1.2, 0.9, 1.0 / 0.8, 1.1, 1.0 / 0.8, 1.3, 1.0 / 0.6, 1.0 / 0.6])
    M = np.array(L.M, dtype=float)
    Lam = np.linalg.inv(M) @ np.diag(s) @ M
    ref = f - Lam @ (f - feq) + (np.eye(9) - Lam / 2) @ F
    t = lambda a: [torch.tensor([[v]], dtype=torch.float64) for v in a]
    out = S.mrt_collide(t(f), t(feq), t(F), list(s))
    assert np.allclose([float(o) for o in out], ref, atol=1e-14)


def test_uniform_state_is_fixed_point():
    for coupled in (True, False):
        prm = _prm(nx=16, ny=16, coupled=coupled, rho1=1.0, rho2=1e-3, mu1=0.01, mu2=1e-4)
        phi = torch.full((16, 16), 0.3, dtype=torch.float64)
        z = torch.zeros_like(phi)
        st = oracle.init_state(phi, z, z, z, prm)
        st1 = oracle.step_once(st, prm)
        assert torch.allclose(st1.fs, st.fs, atol=1e-15, rtol=0)
        if coupled:
            assert torch.allclose(st1.gs, st.gs, atol=1e-15, rtol=0)
