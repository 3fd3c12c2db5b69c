"""Seeded synthetic workloads: parameters and initial fields.

This module holds no step arithmetic.  It only builds the analytic initial
conditions of the paper's benchmarks (tanh interface profiles,
eq:equilibrium_profile; prescribed vortex velocity, Sec. 4.1) and parameter
sets, as plain numbers and float64 numpy arrays.  Both the HIP library (through
its binding) and the CPU oracle consume the same arrays.

Node (i, j) sits at x = i, y = j (lattice units); arrays are indexed [j, i].
Phase +1 is the heavy liquid (rho1), phase -1 the light gas (rho2); a droplet
has phi > 0 inside, a bubble phi < 0 inside.
"""

import dataclasses
import math

import numpy as np

TAU_F = 0.5 + math.sqrt(3.0) / 6.0


def base_params(nx, ny, **kw):
    p = dict(nx=nx, ny=ny, wall_x=False, wall_y=False, coupled=True,
             rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1, sigma=1e-3, W=4.0, M=0.02,
             lam=0.005, tau_f=TAU_F, gx=0.0, gy=0.0, rho_ref=0.0,
             filter_n=11, filter_a=0.5, compact=False, compact_n=5,
             compact_alpha=0.45, K=2, eps=1e-2)
    p.update(kw)
    return p


@dataclasses.dataclass
class Workload:
    name: str
    params: dict
    phi0: np.ndarray
    ux0: np.ndarray
    uy0: np.ndarray
    p0: np.ndarray
    steps: int
    meta: dict = dataclasses.field(default_factory=dict)


def _grid(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return x, y


def drop_field(nx, ny, xc, yc, R, W, inside=1.0, periodic=True):
    """tanh(2(R - r)/W) (inside = +1) or tanh(2(r - R)/W) (inside = -1)."""
    x, y = _grid(nx, ny)
    dx = x - xc
    dy = y - yc
    if periodic:
        dx = dx - nx * np.round(dx / nx)
        dy = dy - ny * np.round(dy / ny)
    r = np.sqrt(dx * dx + dy * dy)
    return np.tanh(inside * 2.0 * (R - r) / W)


def vortex_velocity(nx, ny, U):
    """u = -U sin^2(pi x) sin(2 pi y), v = U sin^2(pi y) sin(2 pi x), x = i/L, y = j/L."""
    x, y = _grid(nx, ny)
    xs = x / nx
    ys = y / ny
    ux = -U * np.sin(np.pi * xs) ** 2 * np.sin(2 * np.pi * ys)
    uy = U * np.sin(np.pi * ys) ** 2 * np.sin(2 * np.pi * xs)
    return ux, uy


def vortex(n=128, U=0.05, steps=1000):
    """Single-vortex deformation of a circle (Sec. 4.1): CH-only, periodic."""
    R = 0.15 * n
    phi = drop_field(n, n, 0.5 * n, 0.75 * n, R, 4.0, inside=1.0)
    ux, uy = vortex_velocity(n, n, U)
    prm = base_params(n, n, coupled=False, sigma=1e-3, lam=0.05, filter_n=0)
    return Workload("vortex", prm, phi, ux, uy, np.zeros_like(phi), steps,
                    dict(R=R, U=U))


def vortex_modulated(L=400, U0=0.02, n_period=2, eta=2.0, lam=0.05, sigma=1e-3, R_frac=0.15,
                     eps=1e-2):
    """Single-vortex deformation as Sec. 4.1 sets it up (eq:velocity): L x L
    periodic, CH only, a circle of radius R_frac L at (0.5L, 0.75L) (the radius
    is not stated; 0.15 L as in the problem the section reproduces), the base
    field u0 = U0 sin^2(pi x) sin(2 pi y), v0 = -U0 sin^2(pi y) sin(2 pi x) with
    x = i/L, y = j/L, modulated by cos(pi t/T), T = n L/U0 (meta["T"]); the
    caller prescribes u0 cos(pi t/T) before each step.  eta = 2 with tau_f =
    1/2 + sqrt(3)/6 gives M = eta c_s^2 (tau_f - 1/2) (eq:mobility)."""
    phi = drop_field(L, L, 0.5 * L, 0.75 * L, R_frac * L, 4.0, inside=1.0)
    x, y = _grid(L, L)
    xs, ys = x / L, y / L
    ux = U0 * np.sin(np.pi * xs) ** 2 * np.sin(2 * np.pi * ys)
    uy = -U0 * np.sin(np.pi * ys) ** 2 * np.sin(2 * np.pi * xs)
    M = eta * (TAU_F - 0.5) / 3.0
    T = n_period * L / U0
    prm = base_params(L, L, coupled=False, sigma=sigma, lam=lam, M=M, filter_n=0, eps=eps)
    return Workload("vortex_modulated", prm, phi, ux, uy, np.zeros_like(phi),
                    int(round(2 * T)), dict(T=T, U0=U0, R=R_frac * L))


def table3_droplet(R=20.0, L=200, original_ch=False, steps=200000, eps=1e-2):
    """The volume test after the Laplace test (Sec. 4.3, Table III): a droplet of
    radius R at the centre of an L x L periodic box, rho1/rho2 = 10/1,
    sigma = 1e-3, tau_f = 0.6 (as printed); the viscosities are not printed:
    nu = 0.01 in both phases; lambda = 0.005, M = 0.02, W = 4, SF-11."""
    phi = drop_field(L, L, 0.5 * L, 0.5 * L, R, 4.0, inside=1.0)
    z = np.zeros_like(phi)
    prm = base_params(L, L, rho1=10.0, rho2=1.0, mu1=0.1, mu2=0.01, sigma=1e-3, tau_f=0.6,
                      original_ch=original_ch, eps=eps)
    return Workload("table3_droplet", prm, phi, z, z.copy(), z.copy(), steps, dict(R=R))


def translating_drop(L=100, U=0.01, lam=0.005, sigma=0.01, steps=4000, R=26.0, W=4.0):
    """Circular drop carried by a uniform velocity (Sec. "Effect of parameter
    lambda"): CH-only on a 3L x L periodic domain (the paper's L x 3L with the
    long side along the motion), centre (L/2, L/2), u = (U, 0)."""
    nx, ny = 3 * L, L
    phi = drop_field(nx, ny, 0.5 * L, 0.5 * L, R, W, inside=1.0)
    ux = np.full_like(phi, U)
    prm = base_params(nx, ny, coupled=False, sigma=sigma, lam=lam, filter_n=0)
    return Workload("translating_drop", prm, phi, ux, np.zeros_like(phi), np.zeros_like(phi),
                    steps, dict(R=R, W=W, xc=0.5 * L, yc=0.5 * L, U=U))


def droplet(n=200, seed=0, steps=20000, sigma=0.01, radii=(20, 25, 30, 35, 40)):
    """Stationary droplet (Laplace law, Sec. 4.3): density ratio 1000, viscosity ratio 100."""
    rng = np.random.default_rng(seed)
    R = float(rng.choice(np.asarray(radii, dtype=np.float64)))
    c = np.array([n / 2, n / 2]) + rng.uniform(-2.0, 2.0, 2)
    phi = drop_field(n, n, c[0], c[1], R, 4.0, inside=1.0)
    z = np.zeros_like(phi)
    prm = base_params(n, n, rho1=1.0, rho2=1e-3, mu1=0.01, mu2=1e-4, sigma=sigma)
    return Workload("droplet", prm, phi, z, z.copy(), z.copy(), steps,
                    dict(R=R, xc=float(c[0]), yc=float(c[1])))


def capillary(nx=128, ny=512, steps=50000, A0_frac=0.01, nu=1e-3, sigma=1e-3,
              rho1=1.0, rho2=1e-3):
    """Capillary wave (Sec. 4.4): heavy layer below, walls in y, periodic in x."""
    x, y = _grid(nx, ny)
    A0 = A0_frac * nx
    y0 = ny / 2 + A0 * np.cos(2 * np.pi * x / nx)
    phi = np.tanh(2.0 * (y0 - y) / 4.0)
    z = np.zeros_like(phi)
    prm = base_params(nx, ny, wall_y=True, rho1=rho1, rho2=rho2, mu1=nu * rho1,
                      mu2=nu * rho2, sigma=sigma)
    return Workload("capillary", prm, phi, z, z.copy(), z.copy(), steps,
                    dict(A0=A0, y0=ny / 2, nu=nu))


def place_bubbles(n, nb, rmin, rmax, W, rng, max_tries=200000):
    """Non-overlapping random circles on a periodic n x n box (min-image distance
    >= R_i + R_j + 2W)."""
    out = []
    tries = 0
    while len(out) < nb:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place bubbles")
        R = rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, 2)
        ok = True
        for (cx, cy, Rj) in out:
            dx = c[0] - cx
            dy = c[1] - cy
            dx -= n * round(dx / n)
            dy -= n * round(dy / n)
            if math.hypot(dx, dy) < R + Rj + 2 * W:
                ok = False
                break
        if ok:
            out.append((float(c[0]), float(c[1]), float(R)))
    return out


def bubbles_field(n, bubbles, W):
    """phi0 = min_i tanh(2(d_i - R_i)/W); evaluated in a box around each bubble
    (beyond d - R > 12 W the tanh rounds to exactly 1.0 in float64)."""
    phi = np.ones((n, n), dtype=np.float64)
    for (cx, cy, R) in bubbles:
        h = int(math.ceil(R + 12 * W)) + 1
        xs = np.arange(int(math.floor(cx)) - h, int(math.floor(cx)) + h + 1)
        ys = np.arange(int(math.floor(cy)) - h, int(math.floor(cy)) + h + 1)
        X, Y = np.meshgrid(xs.astype(np.float64), ys.astype(np.float64), indexing="xy")
        d = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2)
        v = np.tanh(2.0 * (d - R) / W)
        iy = np.mod(ys, n)[:, None]
        ix = np.mod(xs, n)[None, :]
        phi[iy, ix] = np.minimum(phi[iy, ix], v)
    return phi


def bubble_ensemble(n=4096, nb=200, seed=0, steps=2000, rmin=10.0, rmax=60.0,
                    Eo=10.0, Re=35.0, R_ref=35.0, U_g=6.4e-4):
    """Throughput ensemble: gas bubbles in liquid on a periodic box, density ratio
    1000, viscosity ratio 100; gravity from Eo and Re at the reference radius
    (U_g = sqrt(2 g R), Eo = 2 rho1 U_g^2 R / sigma, Re = rho1 U_g 2R / mu1, Sec. 4.5).

    The lattice velocity scale U_g is free; 6.4e-4 keeps the gas-side kinematic
    Laplace pressure sigma/(R rho2) and the buoyancy pressure difference across the
    largest bubble below ~1e-3, the range in which the scheme stays stable at a
    density ratio of 1000 (g = 5.85e-9, sigma = 2.87e-6, mu1 = 1.28e-3)."""
    rng = np.random.default_rng(seed)
    W = 4.0
    bl = place_bubbles(n, nb, rmin, rmax, W, rng)
    phi = bubbles_field(n, bl, W)
    rho1, rho2 = 1.0, 1e-3
    g = U_g * U_g / (2.0 * R_ref)
    sigma = 2.0 * rho1 * U_g * U_g * R_ref / Eo
    mu1 = rho1 * U_g * 2.0 * R_ref / Re
    pm = float(phi.mean())
    rho_ref = rho1 * (1 + pm) / 2 + rho2 * (1 - pm) / 2
    z = np.zeros_like(phi)
    prm = base_params(n, n, rho1=rho1, rho2=rho2, mu1=mu1, mu2=mu1 / 100.0,
                      sigma=sigma, gy=-g, rho_ref=rho_ref)
    return Workload("bubbles", prm, phi, z, z.copy(), z.copy(), steps,
                    dict(nb=nb, bubbles=bl, g=g))


def rising_bubble(nx=256, ny=1024, R=32.0, xc=128.0, yc=128.0, sigma=None, Eo=10.0,
                  Re=35.0, steps=4000, U_g=2e-3, sigma_ref=1e-3, rho_ref=None):
    """Gas bubble rising in liquid in a closed box (walls on all sides), the
    Sec. 4.5 set-up: density ratio 1000, viscosity ratio 100, Eo and Re at the
    initial radius, U_g = sqrt(2 g R).

    U_g is the lattice velocity scale: g = U_g^2/(2R), sigma_0 = 2 rho1 U_g^2 R/Eo,
    mu1 = rho1 U_g 2R/Re.  The default 2e-3 keeps the gas-side kinematic Laplace
    pressure sigma/(R rho2) and the buoyancy pressure difference across the
    bubble (rho1/rho2) g 2R near 1e-3, where the scheme stays stable at a density
    ratio of 1000 for 4000 steps; U_g = None takes g from Eo at sigma_ref
    (g = 2.441e-6, sigma = 1e-3 for R = 32), which diverges within 1000 steps.
    g and the viscosities stay fixed when sigma is varied (sigma = None:
    sigma_0, or sigma_ref without U_g).  rho_ref = None: the liquid density, so
    that F_g = (rho - rho1) g vanishes in the liquid; in a closed box this moves
    the liquid's hydrostatic head into the pressure and leaves the flow
    unchanged, while the gas-side kinematic pressure no longer carries the
    head of the whole box height."""
    rho1, rho2 = 1.0, 1e-3
    if U_g is None:
        g = Eo * sigma_ref / (4.0 * rho1 * R * R)
        U_g = math.sqrt(2.0 * g * R)
        sig0 = sigma_ref
    else:
        g = U_g * U_g / (2.0 * R)
        sig0 = 2.0 * rho1 * U_g * U_g * R / Eo
    sigma = sig0 if sigma is None else sigma
    mu1 = rho1 * U_g * 2.0 * R / Re
    phi = drop_field(nx, ny, xc, yc, R, 4.0, inside=-1.0, periodic=False)
    z = np.zeros_like(phi)
    prm = base_params(nx, ny, wall_x=True, wall_y=True, rho1=rho1, rho2=rho2,
                      mu1=mu1, mu2=mu1 / 100.0, sigma=sigma, gy=-g,
                      rho_ref=rho1 if rho_ref is None else rho_ref)
    return Workload("rising", prm, phi, z, z.copy(), z.copy(), steps,
                    dict(g=g, U_g=U_g, sigma0=sig0, R=R))


# Sec. 4.5, Table IV: (Eo, Re, U_g, rho1/rho2, mu1/mu2)
RISING_TESTS = {1: (10.0, 35.0, 0.0024, 10.0, 10.0), 2: (125.0, 35.0, 0.0019, 1000.0, 100.0)}


def rising_bubble_benchmark(test=1, scale=1.0, steps=None, t_end=3.0):
    """The rising-bubble benchmark of Sec. 4.5: a 1 x 2 domain on 240 x 480 nodes
    (scale = 0.5: 120 x 240), periodic in x, no-slip walls in y, a gas bubble of
    radius 0.25 at (0.5, 0.5), the Eo, Re, U_g and density and viscosity ratios of
    Table IV, U_g = sqrt(2 g R) in lattice units.  rho1 = 1 (lattice), so
    g = U_g^2/(2R), sigma = 2 rho1 U_g^2 R / Eo, mu1 = rho1 U_g 2R / Re; rho_ref =
    rho1 (the liquid's head goes into the pressure).  Time unit: Table IV's own
    units (rho1 = 1000, mu1 = 10, R = 0.25 in a domain of width 1, Re = 35) give
    U_g = Re mu1 / (2 R rho1) = 0.7 per unit of length and time, so one time unit
    is 0.7 L / U_g steps for a domain L nodes wide; `steps` defaults to t_end time
    units."""
    Eo, Re, U_g, rr, mr = RISING_TESTS[test]
    nx, ny = int(round(240 * scale)), int(round(480 * scale))
    R = 0.25 * nx
    rho1 = 1.0
    g = U_g * U_g / (2.0 * R)
    sigma = 2.0 * rho1 * U_g * U_g * R / Eo
    mu1 = rho1 * U_g * 2.0 * R / Re
    phi = drop_field(nx, ny, 0.5 * nx, 0.5 * nx, R, 4.0, inside=-1.0, periodic=False)
    z = np.zeros_like(phi)
    prm = base_params(nx, ny, wall_x=False, wall_y=True, rho1=rho1, rho2=rho1 / rr,
                      mu1=mu1, mu2=mu1 / mr, sigma=sigma, gy=-g, rho_ref=rho1)
    steps_per_time = 0.7 * nx / U_g
    if steps is None:
        steps = int(round(t_end * steps_per_time))
    return Workload(f"rising_test{test}", prm, phi, z, z.copy(), z.copy(), steps,
                    dict(g=g, U_g=U_g, R=R, test=test, steps_per_time=steps_per_time))


def random_smooth(nx, ny, seed, amp=1.0, modes=4):
    """A smooth random periodic field (sum of a few Fourier modes), for tests."""
    rng = np.random.default_rng(seed)
    x, y = _grid(nx, ny)
    f = np.zeros((ny, nx))
    for _ in range(modes):
        kx = rng.integers(0, 4)
        ky = rng.integers(0, 4)
        ph = rng.uniform(0, 2 * np.pi)
        f += rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
    return amp * f / modes
