"""Shared helpers of the GPU tests: run the HIP library and the CPU oracle on the
same seeded inputs and compare."""

import numpy as np
import torch

import oracle
from paper_1812_02459_amd import inputs as I

RTOL64 = 1e-12     # FP64 parity bar: max-norm error relative to the max norm


def relerr(a, b):
    a = a.detach().to("cpu", torch.float64)
    b = b.detach().to("cpu", torch.float64)
    den = float(b.abs().max())
    num = float((a - b).abs().max())
    return num / den if den > 0 else num


def oracle_init(wl, params=None):
    p = dict(wl.params if params is None else params)
    prm = oracle.Params(**p)
    t = lambda a: torch.tensor(a, dtype=torch.float64)
    return oracle.init_state(t(wl.phi0), t(wl.ux0), t(wl.uy0), t(wl.p0), prm), prm


def gpu_sim(wl, params=None, precision=0):
    from paper_1812_02459_amd.binding import Sim
    p = dict(wl.params if params is None else params)
    sim = Sim(p, precision=precision)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    return sim


def droplet_case(nx, ny, seed=0, R=None, **kw):
    """A 1000:1 droplet with a small random velocity and pressure field (all
    phases of the step active from the first step)."""
    rng = np.random.default_rng(seed)
    R = R if R is not None else 0.25 * min(nx, ny)
    xc, yc = nx / 2 + rng.uniform(-2, 2), ny / 2 + rng.uniform(-2, 2)
    periodic = not (kw.get("wall_x") or kw.get("wall_y"))
    phi = I.drop_field(nx, ny, xc, yc, R, 4.0, periodic=periodic)
    ux = 0.01 * I.random_smooth(nx, ny, seed + 1)
    uy = 0.01 * I.random_smooth(nx, ny, seed + 2)
    p = 1e-3 * I.random_smooth(nx, ny, seed + 3)
    if kw.get("wall_y"):
        ux[0, :] = ux[-1, :] = uy[0, :] = uy[-1, :] = 0.0
    prm = I.base_params(nx, ny, rho1=1.0, rho2=1e-3, mu1=0.01, mu2=1e-4, sigma=0.01)
    prm.update(kw)
    return I.Workload("droplet-test", prm, phi, ux, uy, p, 0)
