"""One whole-lattice time step of the fractional-step MRT-LBM (arXiv:1812.02459).

Paper map (section / equation labels of the LaTeX source):
* modified Cahn-Hilliard equation and its split:   Sec. 2.1, eq:final_mCHE,
  eq:step1, eq:step2; free energy eq:free_energy; chemical potential
  eq:chemical; equilibrium profile eq:equilibrium_profile.
* two-phase NS in non-conservative form:           Sec. 2.2, eq:rho,
  eq:surfaceforce, eq:reformNS.
* CH MRT-LBE:   eq:distribution_CH, eq:feq_CH, eq:collison, eq:D2Q9MRT,
  eq:CH_Sf, eq:Fi, eq:mobility, eq:compute_phi.
* FD sub-step:  eq:TVD-3order, eq:fourOrder_FDM.
* NS MRT-LBE:   eq:distribution_NS, eq:geq, eq:Gi, Eq:p, Eq:u, the fixed-point
  velocity iteration (text after eq:Fmu), eq:dynamic_vis, eq:dicretized,
  eq:filter (+ App. B).

Phase order of one step n -> n+1 (the paper does not spell it out; this is the
order its text implies):
  1. stream f*, g*; gather phi_bar = sum f, p = c_s^2 sum g, j = sum g c
  2. FD sub-step: phi^{n+1} = TVD-RK3(phi_bar) with L = div J_d
  3. properties from phi^{n+1}; 4. K fixed-point iterations of u = j + F(u)/(2 rho)
  5. selective filter on (p, u)  6. MRT collision of f and g at n+1
  7. keep the filtered u as u~^n for the next step's d_t u.

Readings (places where the paper is silent, ambiguous or garbled):
R1  lambda (Sec. 4.2 "lambda in eq:final_mCHE", absent from it): J_d = lambda*J_phi + q.
R2  n = grad phi/|grad phi| is regularised: |G|_eps = sqrt(|G|^2 + eps^2) in n
    and in the first factor of J_phi.  Where |G| < eps the correction is a
    diffusion with coefficient lambda (1 - c/eps), c = 2(1 - phi^2)/W, so eps
    sets how close to +-1 the bulk may sit before the term turns
    anti-diffusive; eps = 1e-2 (2% of the interface gradient 2/W at W = 4)
    keeps the sharpening inside the interface (|phi| < 0.99).  With
    eps = 1e-9 the bulk of a light phase fills with grid-scale noise and 1000:1
    gas bubbles diverge.
R3  mu inside the FD sub-step uses the isotropic Laplacian of eq:dicretized;
    the first derivatives (grad phi, grad mu, divergence) use eq:fourOrder_FDM.
R4  eq:fourOrder_FDM's typos (i+2dx, repeated y-2dy, j+dy) read as the standard
    [P(-2) - 8P(-1) + 8P(+1) - P(+2)] / 12 in x and in y.
R5  weights omega_{5..8} = 1/36 (the paper prints omega_{1..8}).
R6  S^f = (1,1,1,1/tau_f,1,1/tau_f,1,1,1) (only s3, s5 given); s0 = 1 makes the
    collision set sum f* = phi^{n+1}, which carries the FD correction back
    into the populations.
R7  S^g = (1,1,1,1,1,1,1,1/tau_g,1/tau_g) (only s7, s8 given); s0 = s3 = s5 = 1
    carry the filtered p, u into the populations; s1 = 1 (bulk viscosity 1/6).
R8  eq:Gi's u(F - grad p)/rho read as u b with b = F/rho - grad p, the form the
    first-order momentum balance of App. A needs to cancel d_t1(uu) when p is
    the kinematic pressure.
R9  F_nu uses the isotropic FD velocity gradient (the paper allows FD instead of
    the moment formula eq:Fmu).
R10 the implicit velocity runs a fixed number K of iterations from u^0 = u~^n
    (the paper iterates to an unstated threshold zeta); the residual is
    reported.
R11 filter: unsplit (both directions read unfiltered inputs), on chi = (p, u)
    only, SF-11 with a = 0.5 by default (Sec. 4.3).
R12 d_t u in eq:Fi is (u~^{n+1} - u~^n)/dt; u.grad u uses the isotropic gradient.
R13 rho, dynamic viscosity and tau_g are evaluated from clamp(phi, -1, 1);
    phi itself is never clamped (clipping breaks conservation, Sec. 1).
    grad rho (in F_p and F_nu) is the isotropic gradient of that density field,
    so that grad rho / rho stays bounded where phi leaves [-1, 1] in the light
    phase (with (rho1-rho2)/2 grad phi instead, a 1000:1 droplet diverges
    within ~80 steps); J keeps d rho/d phi = (rho1 - rho2)/2 (Sec. 2.2).
R14 walls: half-way bounce-back for f and g; ghost mirror for stencils with
    phi, mu, p even and u odd.
R15 initial state: f* = f^eq(phi0, mu(phi0), u0), g* = g^eq(p0, u0), u~ = u0.
R16 gravity enters as F_g = (rho - rho_ref) g; rho_ref = mean density on a fully
    periodic box (constant, since sum phi is conserved), 0 with walls.
R17 eta = M / (c_s^2 (tau_f - 1/2)) from eq:mobility, eta being "adjustable for a
    given mobility".
R18 CH-only mode (prescribed velocity, no hydrodynamics): u~ = the prescribed u;
    d_t u in eq:Fi is the backward difference of the prescribed velocities of
    consecutive steps (R12's difference), 0 for a velocity held fixed.
R19 "original CH" (Sec. 4.1-4.3 comparisons, lambda = 0) means no FD sub-step at all.
R20 strain rate from the moments (eq:Fmu, an option; R9 is the default).  The
    printed formula is garbled (f for g; F for the F - grad p of eq:Gi) and is
    re-derived here from App. A's first-order balances of m_1, m_7 and m_8
    (eq:t2momentum_auxilliary, with d_t1 p = -c_s^2 div u and d_t1 u = b + O(u^2),
    b = F/rho - grad p per R8): with A_k = m_k(g) - m_k^eq + G~_k/2 of the
    pre-collision g,
        div u = -(s_1/2) A_1,  d_x u_x - d_y u_y = -(3/2) s_7 A_7,
        d_x u_y + d_y u_x = -3 s_8 A_8,
    m_1^eq = -6p + 3|u|^2, m_7^eq = u_x^2 - u_y^2, m_8^eq = u_x u_y,
    G~_1/2 = 3 b.u, G~_7/2 = b_x u_x - b_y u_y, G~_8/2 = (b_x u_y + b_y u_x)/2.
    Inside F the strain rate enters F_nu itself, so the b of these corrections
    is the one of the other force parts (F - F_nu)/rho - grad p (with R21:
    (F - F_nu - grad p)/rho).
R21 literal eq:Gi (an option for the study of R8): b = (F - grad p)/rho.
"""

import dataclasses
from typing import Optional

import torch

from .lattice import C, W, OPP, M as MRT, MM_DIAG_INV, FILTER_D
from .ops import ext, crop, iso_grad, iso_lap, d4x, d4y, selective_filter, sqrt
from . import compact

DT = torch.float64


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    wall_x: bool = False
    wall_y: bool = False
    coupled: bool = True          # False: CH-only with a prescribed velocity
    rho1: float = 1.0             # phase phi = +1
    rho2: float = 1.0             # phase phi = -1
    mu1: float = 0.1
    mu2: float = 0.1
    sigma: float = 1e-3
    W: float = 4.0                # interface width
    M: float = 0.02               # mobility
    lam: float = 0.005            # lambda (R1)
    tau_f: float = 0.5 + 3 ** 0.5 / 6
    gx: float = 0.0
    gy: float = 0.0
    rho_ref: float = 0.0
    filter_n: int = 11            # 0: off; 5, 7, 9, 11: explicit SF-n (App. B)
    filter_a: float = 0.5
    compact: bool = False         # compact (tridiagonal) selective filter instead
    compact_n: int = 5
    compact_alpha: float = 0.45
    K: int = 2                    # velocity fixed-point iterations (R10)
    s_f: tuple = (1.0, 1.0, 1.0, None, 1.0, None, 1.0, 1.0, 1.0)
    s_g: tuple = (1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, None, None)
    eps: float = 1e-2             # |grad phi| regularisation (R2)
    original_ch: bool = False     # no FD sub-step: the original convective CH (Sec. 4.2)
    strain_moments: bool = False  # F_nu's strain rate from the moments of g (R20, eq:Fmu)
    gi_literal: bool = False      # eq:Gi as printed, b = (F - grad p)/rho (R21)

    # derived constants, Sec. 2.1 and eq:mobility
    @property
    def kappa(self):
        return 3 * self.sigma * self.W / 8

    @property
    def beta(self):
        return 3 * self.sigma / (4 * self.W)

    @property
    def eta(self):
        return (3.0 * self.M) / (self.tau_f - 0.5)


@dataclasses.dataclass
class State:
    fs: torch.Tensor                    # (9, ny, nx) post-collision f*
    gs: Optional[torch.Tensor]          # (9, ny, nx) post-collision g* (coupled)
    uo: torch.Tensor                    # (2, ny, nx) filtered velocity u~^n
    n: int = 0
    # fields of the last step, for reporting and per-phase comparison
    phi: Optional[torch.Tensor] = None
    p: Optional[torch.Tensor] = None
    phibar: Optional[torch.Tensor] = None
    praw: Optional[torch.Tensor] = None
    j: Optional[torch.Tensor] = None
    uK: Optional[torch.Tensor] = None
    resid: Optional[float] = None
    # CH-only: the velocity the last step used, when set_velocity has replaced it
    up: Optional[torch.Tensor] = None


# ----------------------------------------------------------------------------
# pointwise pieces
# ----------------------------------------------------------------------------

def _cdot(i, ax, ay):
    """c_i . a with zero components skipped (c entries are 0 or +-1)."""
    cx, cy = C[i]
    if cx == 0 and cy == 0:
        return torch.zeros_like(ax)
    if cy == 0:
        return cx * ax
    if cx == 0:
        return cy * ay
    return cx * ax + cy * ay


def chem_pot(P, prm):
    """mu_phi = 4 beta (phi^3 - phi) - kappa lap(phi), eq:chemical.  Shrinks halo by 1."""
    P0 = crop(P, 1, 0)
    return (4 * prm.beta) * ((P0 * P0) * P0 - P0) - prm.kappa * iso_lap(P)


def f_eq(phi, mu, ux, uy, prm):
    """CH equilibrium, eq:feq_CH."""
    eta = prm.eta
    usq = ux * ux + uy * uy
    out = []
    for i in range(9):
        if i == 0:
            out.append((phi + ((W[0] - 1) * eta) * mu) - ((W[0] * phi) * usq) * 1.5)
        else:
            cu = _cdot(i, ux, uy)
            inner = ((cu * 3.0) + ((cu * cu) * 4.5)) - usq * 1.5
            out.append((W[i] * eta) * mu + (W[i] * phi) * inner)
    return out


def g_eq(p, ux, uy):
    """Velocity-based pressure equilibrium, eq:geq."""
    usq = ux * ux + uy * uy
    out = []
    for i in range(9):
        cu = _cdot(i, ux, uy)
        out.append(W[i] * (((p * 3.0 + cu * 3.0) + (cu * cu) * 4.5) - usq * 1.5))
    return out


def src_f(phi, ax, ay):
    """CH source, eq:Fi: F_i = w_i phi c_i.(d_t u + u.grad u) / c_s^2."""
    out = [torch.zeros_like(phi)]
    for i in range(1, 9):
        out.append(((W[i] * phi) * _cdot(i, ax, ay)) * 3.0)
    return out


def src_g(Fx, Fy, rho, ux, uy, bx, by):
    """NS source, eq:Gi with reading R8 (b = F/rho - grad p):
    G_i = w_i [ c_i.(F/rho) / c_s^2 + (u b):(c_i c_i - c_s^2 I) / c_s^4 ]."""
    Frx = Fx / rho
    Fry = Fy / rho
    ub = ux * bx + uy * by
    out = []
    for i in range(9):
        cF = _cdot(i, Frx, Fry)
        cu = _cdot(i, ux, uy)
        cb = _cdot(i, bx, by)
        out.append(W[i] * ((cF * 3.0) + ((cu * cb) - ub / 3.0) * 9.0))
    return out


def m_apply(v):
    """m_k = sum_j M_kj v_j (eq:D2Q9MRT), accumulated in j order, zeros skipped."""
    out = []
    for k in range(9):
        acc = 0
        for j in range(9):
            if MRT[k][j] != 0:
                acc = acc + MRT[k][j] * v[j]
        out.append(acc)
    return out


def minv_apply(m):
    """v = M^{-1} m with M^{-1} = M^T diag(1/(M M^T)_kk); sums in k order."""
    sc = [m[k] * MM_DIAG_INV[k] for k in range(9)]
    out = []
    for j in range(9):
        acc = 0
        for k in range(9):
            if MRT[k][j] != 0:
                acc = acc + MRT[k][j] * sc[k]
        out.append(acc)
    return out


def mrt_collide(f, feq, F, s):
    """eq:distribution_CH / eq:distribution_NS right-hand side with
    Lambda = M^{-1} S M (eq:collison):
        f* = f - Lambda (f - f^eq) + (I - Lambda/2) F
           = f + M^{-1} [ (I - S/2) M F - S M (f - f^eq) ]."""
    d = [f[i] - feq[i] for i in range(9)]
    md = m_apply(d)
    mF = m_apply(F)
    r = [(1.0 - s[k] * 0.5) * mF[k] - s[k] * md[k] for k in range(9)]
    corr = minv_apply(r)
    return [f[i] + corr[i] for i in range(9)]


# ----------------------------------------------------------------------------
# streaming and moments
# ----------------------------------------------------------------------------

def stream(fs, prm):
    """f_i(x, t+1) = f*_i(x - c_i, t) (left side of eq:distribution_CH/NS), with
    half-way bounce-back f_i(x) = f*_opp(i)(x) where x - c_i lies beyond a wall (R14)."""
    ny, nx = fs.shape[1], fs.shape[2]
    ys = torch.arange(ny)[:, None]
    xs = torch.arange(nx)[None, :]
    out = []
    for i in range(9):
        cx, cy = C[i]
        fi = torch.roll(fs[i], shifts=(cy, cx), dims=(0, 1))
        outside = torch.zeros(ny, nx, dtype=torch.bool)
        if prm.wall_x and cx != 0:
            outside = outside | ((xs - cx) < 0) | ((xs - cx) >= nx)
        if prm.wall_y and cy != 0:
            outside = outside | ((ys - cy) < 0) | ((ys - cy) >= ny)
        if bool(outside.any()):
            fi = torch.where(outside, fs[OPP[i]], fi)
        out.append(fi)
    return out


def gather(f, g):
    """phi_bar = sum f_i (eq:compute_phi); p = c_s^2 sum g_i (Eq:p); j = sum g_i c_i
    (the first part of Eq:u)."""
    phibar = f[0]
    for i in range(1, 9):
        phibar = phibar + f[i]
    if g is None:
        return phibar, None, None, None
    sg = g[0]
    for i in range(1, 9):
        sg = sg + g[i]
    praw = sg / 3.0
    jx = 0
    jy = 0
    for i in range(9):
        cx, cy = C[i]
        if cx != 0:
            jx = jx + cx * g[i]
        if cy != 0:
            jy = jy + cy * g[i]
    return phibar, praw, jx, jy


# ----------------------------------------------------------------------------
# FD sub-step (eq:step2 with eq:TVD-3order)
# ----------------------------------------------------------------------------

def fd_rhs(phi, prm):
    """L(phi*) = div J_d with J_d = lambda J_phi + q (eq:final_mCHE, R1-R4).

    J_phi = (|grad phi| - 2(1 - phi^2)/W) n,   q = (-M grad mu . n) n,
    n = grad phi / |grad phi|_eps.  Derivatives: eq:fourOrder_FDM.
    """
    P = ext(phi, 5, prm.wall_x, prm.wall_y)           # halo 5
    mu = chem_pot(P, prm)                              # halo 4
    Gx = crop(d4x(P), 3, 2)                            # halo 2
    Gy = crop(d4y(P), 3, 2)
    Mx = d4x(mu)                                       # halo 2
    My = d4y(mu)
    ph = crop(P, 5, 2)
    mag = sqrt((Gx * Gx + Gy * Gy) + prm.eps * prm.eps)
    nx_ = Gx / mag
    ny_ = Gy / mag
    cW = 2 * (1 - ph * ph) / prm.W
    Jpx = (mag - cW) * nx_
    Jpy = (mag - cW) * ny_
    s = Mx * nx_ + My * ny_
    negM = -prm.M
    qx = (negM * s) * nx_
    qy = (negM * s) * ny_
    Jdx = prm.lam * Jpx + qx
    Jdy = prm.lam * Jpy + qy
    return d4x(Jdx) + d4y(Jdy)                         # halo 0


def rk3(phibar, L):
    """Third-order TVD Runge-Kutta, eq:TVD-3order, dt = 1."""
    phi1 = phibar + L(phibar)
    phi2 = 0.75 * phibar + 0.25 * (phi1 + L(phi1))
    return phibar / 3.0 + 2.0 * (phi2 + L(phi2)) / 3.0


# ----------------------------------------------------------------------------
# hydrodynamic forces (Sec. 2.2, eq:reformNS) on the isotropic stencils
# ----------------------------------------------------------------------------

def properties(ph, prm):
    """rho (eq:rho), dynamic viscosity (eq:dynamic_vis), nu = mu/rho, from the
    clamped order parameter (R13)."""
    phc = torch.clamp(ph, -1.0, 1.0)
    rho = prm.rho1 * (1 + phc) / 2 + prm.rho2 * (1 - phc) / 2
    muv = prm.mu1 * (1 + phc) / 2 + prm.mu2 * (1 - phc) / 2
    return rho, muv / rho


def strain_from_moments(g, p, ux, uy, bx, by, nu, prm):
    """grad u + grad u^T from the non-equilibrium moments of the pre-collision g
    (eq:Fmu as re-derived in R20); returns (S_xx, S_xy, S_yy)."""
    m = m_apply(g)
    s1 = prm.s_g[1]
    s7 = 1.0 / (nu * 3.0 + 0.5)                 # s_7 = s_8 = 1/tau_g (eq:dynamic_vis)
    A1 = (m[1] - ((-6.0) * p + 3.0 * (ux * ux + uy * uy))) + 3.0 * (bx * ux + by * uy)
    A7 = (m[7] - (ux * ux - uy * uy)) + (bx * ux - by * uy)
    A8 = (m[8] - ux * uy) + 0.5 * (bx * uy + by * ux)
    div = (-0.5 * s1) * A1
    D = (-1.5 * s7) * A7
    return div + D, (-3.0 * s7) * A8, div - D


def forces(phi, p, ux, uy, prm, g=None):
    """F = F_p + F_s + F_nu + F_m + F_g (eq:reformNS, eq:surfaceforce, Sec. 2.2).

    phi: order parameter (no halo), p: pressure (no halo), ux/uy: velocity
    (no halo).  Returns a dict with F, rho, nu, grad u and mu_phi at the nodes.
    With prm.strain_moments, the strain rate of F_nu comes from the moments of
    the pre-collision populations g (R20) instead of the velocity's stencil.
    """
    wx, wy = prm.wall_x, prm.wall_y
    P2 = ext(phi, 2, wx, wy)
    U1x = ext(ux, 1, wx, wy, odd=True)
    U1y = ext(uy, 1, wx, wy, odd=True)
    rho, nu = properties(phi, prm)
    # chemical potential on halo 1, its isotropic gradient at the nodes
    mup = chem_pot(P2, prm)
    dmx, dmy = iso_grad(mup)
    cJ = (prm.rho1 - prm.rho2) / 2 * prm.M
    Jx = cJ * dmx                                      # J = (d rho/d phi) M grad mu
    Jy = cJ * dmy
    # surface force, eq:surfaceforce: kappa div(|grad phi|^2 I - grad phi grad phi)
    px, py = iso_grad(P2)                              # halo 1
    dxyy, _ = iso_grad(py * py)
    dxxy, dyxy = iso_grad(px * py)
    _, dyxx = iso_grad(px * px)
    Fsx = prm.kappa * (dxyy - dyxy)
    Fsy = prm.kappa * (dyxx - dxxy)
    # grad rho: isotropic gradient of the density field (R13)
    rho1h, _ = properties(crop(P2, 2, 1), prm)
    grx, gry = iso_grad(rho1h)
    duxx, duxy = iso_grad(U1x)                         # d ux/dx, d ux/dy
    duyx, duyy = iso_grad(U1y)
    Fpx = -p * grx
    Fpy = -p * gry
    Fmx = Jx * duxx + Jy * duxy
    Fmy = Jx * duyx + Jy * duyy
    Fgx = (rho - prm.rho_ref) * prm.gx
    Fgy = (rho - prm.rho_ref) * prm.gy
    if prm.strain_moments and g is not None:
        dpx, dpy = iso_grad(ext(p, 1, wx, wy))
        Frx = ((Fpx + Fsx) + Fmx) + Fgx
        Fry = ((Fpy + Fsy) + Fmy) + Fgy
        if prm.gi_literal:
            brx = (Frx - dpx) / rho
            bry = (Fry - dpy) / rho
        else:
            brx = Frx / rho - dpx
            bry = Fry / rho - dpy
        Sxx, Sxy, Syy = strain_from_moments(g, p, ux, uy, brx, bry, nu, prm)
    else:
        Sxx = duxx + duxx
        Sxy = duyx + duxy
        Syy = duyy + duyy
    Fnx = nu * (Sxx * grx + Sxy * gry)
    Fny = nu * (Sxy * grx + Syy * gry)
    Fx = (((Fpx + Fsx) + Fnx) + Fmx) + Fgx
    Fy = (((Fpy + Fsy) + Fny) + Fmy) + Fgy
    return dict(Fx=Fx, Fy=Fy, rho=rho, nu=nu, mu=mup[1:-1, 1:-1], Jx=Jx, Jy=Jy,
                grx=grx, gry=gry,
                duxx=duxx, duxy=duxy, duyx=duyx, duyy=duyy)


def velocity_iteration(phi, praw, jx, jy, u0x, u0y, prm, g=None):
    """u = sum g c + F(u) dt/(2 rho) (Eq:u), solved by K fixed-point sweeps (R10);
    g: the pre-collision populations (the strain rate of R20)."""
    ux, uy = u0x, u0y
    prevx, prevy = ux, uy
    for _ in range(prm.K):
        fr = forces(phi, praw, ux, uy, prm, g=g)
        prevx, prevy = ux, uy
        ux = jx + fr["Fx"] / (2 * fr["rho"])
        uy = jy + fr["Fy"] / (2 * fr["rho"])
    num = float((ux - prevx).abs().sum() + (uy - prevy).abs().sum())
    den = float(prevx.abs().sum() + prevy.abs().sum())
    resid = num / den if den > 0 else 0.0
    return ux, uy, resid


def filter_fields(p, ux, uy, prm):
    """Selective filter on chi = (p, u) (eq:filter, R11) or its compact variant."""
    wx, wy = prm.wall_x, prm.wall_y
    if prm.compact:
        a = prm.filter_a
        return (compact.filter2d(p, prm.compact_n, prm.compact_alpha, a, wx, wy, odd=False),
                compact.filter2d(ux, prm.compact_n, prm.compact_alpha, a, wx, wy, odd=True),
                compact.filter2d(uy, prm.compact_n, prm.compact_alpha, a, wx, wy, odd=True))
    if prm.filter_n == 0:
        return p, ux, uy
    d = FILTER_D[prm.filter_n]
    h = len(d) - 1
    a = prm.filter_a
    return (selective_filter(ext(p, h, wx, wy), d, a),
            selective_filter(ext(ux, h, wx, wy, odd=True), d, a),
            selective_filter(ext(uy, h, wx, wy, odd=True), d, a))


def _s_f(prm):
    s = list(prm.s_f)
    s[3] = 1.0 / prm.tau_f
    s[5] = 1.0 / prm.tau_f
    return s


def _s_g(prm, nu):
    s = list(prm.s_g)
    tau_g = nu * 3.0 + 0.5                     # tau_g = mu/(rho c_s^2) + 1/2
    sv = 1.0 / tau_g
    s[7] = sv
    s[8] = sv
    return s


def accel(ux, uy, uox, uoy, prm):
    """Material acceleration d_t u + (u.grad) u of eq:Fi (R12)."""
    U1x = ext(ux, 1, prm.wall_x, prm.wall_y, odd=True)
    U1y = ext(uy, 1, prm.wall_x, prm.wall_y, odd=True)
    duxx, duxy = iso_grad(U1x)
    duyx, duyy = iso_grad(U1y)
    ax = (ux - uox) + (ux * duxx + uy * duxy)
    ay = (uy - uoy) + (ux * duyx + uy * duyy)
    return ax, ay


def collide(f, g, phi, p, ux, uy, uox, uoy, prm):
    """MRT collision of f and g at time n+1 (eq:distribution_CH, eq:distribution_NS)."""
    wx, wy = prm.wall_x, prm.wall_y
    ax, ay = accel(ux, uy, uox, uoy, prm)
    mu = chem_pot(ext(phi, 1, wx, wy), prm)
    fst = mrt_collide(f, f_eq(phi, mu, ux, uy, prm), src_f(phi, ax, ay), _s_f(prm))
    if g is None:
        return fst, None
    fr = forces(phi, p, ux, uy, prm, g=g)
    dpx, dpy = iso_grad(ext(p, 1, wx, wy))
    rho = fr["rho"]
    if prm.gi_literal:
        bx = (fr["Fx"] - dpx) / rho
        by = (fr["Fy"] - dpy) / rho
    else:
        bx = fr["Fx"] / rho - dpx
        by = fr["Fy"] / rho - dpy
    gst = mrt_collide(g, g_eq(p, ux, uy),
                      src_g(fr["Fx"], fr["Fy"], rho, ux, uy, bx, by),
                      _s_g(prm, fr["nu"]))
    return fst, gst


# ----------------------------------------------------------------------------
# driver
# ----------------------------------------------------------------------------

def init_state(phi0, ux0, uy0, p0, prm):
    """Equilibrium initial populations (R15)."""
    phi0 = phi0.to(DT)
    ux0 = ux0.to(DT)
    uy0 = uy0.to(DT)
    mu = chem_pot(ext(phi0, 1, prm.wall_x, prm.wall_y), prm)
    fs = torch.stack(f_eq(phi0, mu, ux0, uy0, prm))
    gs = None
    if prm.coupled:
        gs = torch.stack(g_eq(p0.to(DT), ux0, uy0))
    return State(fs=fs, gs=gs, uo=torch.stack([ux0, uy0]), n=0,
                 phi=phi0.clone(), p=p0.to(DT).clone())


def step(st, prm):
    """Advance the state by one time step; returns a new State."""
    f = stream(st.fs, prm)
    g = stream(st.gs, prm) if prm.coupled else None
    phibar, praw, jx, jy = gather(f, g)
    phi = phibar if prm.original_ch else rk3(phibar, lambda q: fd_rhs(q, prm))
    uox, uoy = st.uo[0], st.uo[1]
    if not prm.coupled:
        prev = st.uo if st.up is None else st.up
        fst, _ = collide(f, None, phi, None, uox, uoy, prev[0], prev[1], prm)
        return State(fs=torch.stack(fst), gs=None, uo=st.uo, n=st.n + 1,
                     phi=phi, phibar=phibar)
    uKx, uKy, resid = velocity_iteration(phi, praw, jx, jy, uox, uoy, prm, g=g)
    pt, utx, uty = filter_fields(praw, uKx, uKy, prm)
    fst, gst = collide(f, g, phi, pt, utx, uty, uox, uoy, prm)
    return State(fs=torch.stack(fst), gs=torch.stack(gst), uo=torch.stack([utx, uty]),
                 n=st.n + 1, phi=phi, p=pt, phibar=phibar, praw=praw,
                 j=torch.stack([jx, jy]), uK=torch.stack([uKx, uKy]), resid=resid)


def set_velocity(st, ux, uy):
    """CH-only mode: prescribe the velocity of the following steps (Sec. 4.1's
    vortex is modulated in time, cos(pi t / T)).  The next step's d_t u is the
    new velocity minus the one the last step used (R18)."""
    prev = st.uo if st.up is None else st.up
    return dataclasses.replace(st, uo=torch.stack([ux.to(DT), uy.to(DT)]), up=prev)


def run(st, prm, nsteps):
    for _ in range(nsteps):
        st = step(st, prm)
    return st
