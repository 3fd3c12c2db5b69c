"""Closed-form pins of the oracle's force terms, acceleration and flux correction.

On polynomial fields the isotropic stencils are exact (quadratics for the
gradient), so the discrete terms must equal their continuum definitions
(Sec. 2.2, eq:surfaceforce, eq:reformNS; eq:Fi):
* F_p = -p grad rho, F_nu = nu (grad u + grad u^T) . grad rho, F_g = (rho - rho_ref) g;
* F_m = (J . grad) u -- the orientation of the contraction is what is pinned;
* F_s = kappa div(|grad phi|^2 I - grad phi grad phi) = kappa (H grad phi - tr(H) grad phi)
  for a quadratic phi with Hessian H;
* (u . grad) u of the CH source;
* the flux correction q removes the normal diffusive flux, which is what keeps the
  volume of a small droplet (Table III: "present" 0 %, original CH shrinks).
"""

import numpy as np
import torch

import oracle
from oracle import step as S
from oracle import diagnostics as D
from paper_1812_02459_amd import inputs as I

N = 16
B = 3          # border excluded: periodic ghosts break polynomial fields


def _xy():
    y, x = torch.meshgrid(torch.arange(N, dtype=torch.float64),
                          torch.arange(N, dtype=torch.float64), indexing="ij")
    return x - N / 2, y - N / 2


def _inner(a):
    return a[B:-B, B:-B]


def _prm(**kw):
    base = dict(nx=N, ny=N, rho1=1.0, rho2=0.2, mu1=0.05, mu2=0.01, sigma=0.0,
                M=0.03, gx=1e-4, gy=-2e-4, rho_ref=0.3)
    base.update(kw)
    return oracle.Params(**base)


def _linear_u(x, y):
    A = np.array([[0.3, -0.7], [0.5, 0.2]]) * 1e-3     # A[a, b] = d_a u_b
    ux = A[0, 0] * x + A[1, 0] * y + 1e-3
    uy = A[0, 1] * x + A[1, 1] * y - 2e-3
    return ux, uy, A


def test_pressure_viscous_gravity_terms():
    prm = _prm()
    x, y = _xy()
    phi = 0.05 + 0.01 * x - 0.02 * y
    ux, uy, A = _linear_u(x, y)
    p = torch.full_like(x, 0.013)
    fr = S.forces(phi, p, ux, uy, prm)
    rho = prm.rho1 * (1 + phi) / 2 + prm.rho2 * (1 - phi) / 2
    mu = prm.mu1 * (1 + phi) / 2 + prm.mu2 * (1 - phi) / 2
    nu = mu / rho
    gr = (prm.rho1 - prm.rho2) / 2 * np.array([0.01, -0.02])
    Ssym = A + A.T
    Fnu = Ssym @ gr
    Fx = -0.013 * gr[0] + nu * Fnu[0] + (rho - prm.rho_ref) * prm.gx
    Fy = -0.013 * gr[1] + nu * Fnu[1] + (rho - prm.rho_ref) * prm.gy
    assert torch.allclose(_inner(fr["Fx"]), _inner(Fx), atol=1e-15, rtol=1e-12)
    assert torch.allclose(_inner(fr["Fy"]), _inner(Fy), atol=1e-15, rtol=1e-12)


def test_momentum_flux_term_orientation():
    prm = _prm(sigma=0.02, gx=0.0, gy=0.0)
    x, y = _xy()
    phi = 0.05 + 0.01 * x - 0.02 * y + 0.002 * x * y
    ux, uy, A = _linear_u(x, y)
    z = torch.zeros_like(x)
    f1 = S.forces(phi, z, ux, uy, prm)
    f0 = S.forces(phi, z, z, z, prm)
    rho = f1["rho"]
    gr = torch.stack([f1["grx"], f1["gry"]])
    Ssym = torch.tensor(A + A.T)
    Fnu = f1["nu"] * torch.einsum("ab,byx->ayx", Ssym, gr)
    J = torch.stack([f1["Jx"], f1["Jy"]])
    Fm = torch.einsum("ab,ayx->byx", torch.tensor(A), J)   # (J.grad) u_b = sum_a J_a d_a u_b
    dF = torch.stack([f1["Fx"] - f0["Fx"], f1["Fy"] - f0["Fy"]])
    assert torch.allclose(_inner(dF[0]), _inner(Fnu[0] + Fm[0]), atol=1e-17, rtol=1e-10)
    assert torch.allclose(_inner(dF[1]), _inner(Fnu[1] + Fm[1]), atol=1e-17, rtol=1e-10)
    assert float(Fm[:, B:-B, B:-B].abs().max()) > 1e-10      # the term is exercised


def test_surface_force_quadratic_phi():
    prm = _prm(sigma=0.03, gx=0.0, gy=0.0)
    x, y = _xy()
    a, b, c, d, e = 0.001, -0.002, 0.0015, 0.01, 0.02
    phi = a * x * x + b * x * y + c * y * y + d * x + e * y
    z = torch.zeros_like(x)
    fr = S.forces(phi, z, z, z, prm)
    px = 2 * a * x + b * y + d
    py = b * x + 2 * c * y + e
    H = np.array([[2 * a, b], [b, 2 * c]])
    Fsx = prm.kappa * ((H[0, 0] * px + H[0, 1] * py) - np.trace(H) * px)
    Fsy = prm.kappa * ((H[1, 0] * px + H[1, 1] * py) - np.trace(H) * py)
    assert torch.allclose(_inner(fr["Fx"]), _inner(Fsx), atol=1e-18, rtol=1e-10)
    assert torch.allclose(_inner(fr["Fy"]), _inner(Fsy), atol=1e-18, rtol=1e-10)


def test_material_acceleration():
    prm = _prm()
    x, y = _xy()
    ux, uy, A = _linear_u(x, y)
    uox, uoy = 0.9 * ux, 1.1 * uy
    ax, ay = S.accel(ux, uy, uox, uoy, prm)
    U = torch.stack([ux, uy])
    adv = torch.einsum("ayx,ab->byx", U, torch.tensor(A))   # sum_a u_a d_a u_b
    assert torch.allclose(_inner(ax), _inner(ux - uox + adv[0]), atol=1e-18, rtol=1e-12)
    assert torch.allclose(_inner(ay), _inner(uy - uoy + adv[1]), atol=1e-18, rtol=1e-12)


def test_flux_correction_keeps_small_droplet_volume():
    n, R = 40, 6.0
    phi = torch.tensor(I.drop_field(n, n, 20.3, 19.6, R, 4.0))
    z = torch.zeros_like(phi)
    vols = {}
    for orig in (True, False):
        prm = oracle.Params(**I.base_params(n, n, coupled=False, sigma=0.01, M=0.1,
                                            lam=0.005, original_ch=orig))
        st = oracle.run(oracle.init_state(phi, z, z, z, prm), prm, 2000)
        vols[orig] = (D.volume(st.phi), float(st.phi.max()))
    v0 = D.volume(phi)
    assert vols[False][0] == v0                  # present method: volume kept
    assert vols[True][0] < v0 - 1                # original CH: the droplet shrinks
    assert vols[False][1] < 1.0 and vols[True][1] > 1.0   # only the correction keeps phi <= 1
