"""FP64 parity with the oracle at the walled benchmark sizes, the prescribed
time-modulated velocity of the CH-only mode, and the non-finite-state check.

* the capillary wave's lattice (Sec. 4.4: 128 x 512, walls in y) and the
  rising bubble's (Sec. 4.5: 256 x 1024, walls on all sides), and a walled
  520 x 300 droplet: enough tiles that every kernel runs its production
  launch shape with wall ghosts (the smaller parity cases run the
  short-tile shapes of lattices with fewer than 64 tiles); 1, 5 and 20
  steps, every field within 1e-12 of the oracle's;
* one FP32 step on the same lattices against the FP64 oracle, with the
  per-step FP32 bars of the full-size window test;
* the single vortex of Sec. 4.1 with its time modulation cos(pi t / T),
  the velocity set before every step through lbm2p_set_velocity;
* a NaN or Inf in phi0 reaches the state and lbm2p_volume reports it.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1812_02459_amd import inputs as I

from gpu_common import RTOL64, relerr, oracle_init, gpu_sim

pytestmark = pytest.mark.gpu

# per-step FP32 bars, as in the full-size window test (errors over each field's
# maximum): unit roundoff x ~30 roundings, x rho1/rho2 for g and u
RTOL32_STEP = {"f": 2e-6, "phi": 2e-6, "p": 2e-6, "g": 6e-5, "u": 6e-5}


def _perturbed(wl, seed, amp_u=1e-3, amp_p=1e-4):
    """The workload with a smooth random velocity and pressure on top (every
    term of the step active from the first step)."""
    nx, ny = wl.params["nx"], wl.params["ny"]
    ux = wl.ux0 + amp_u * I.random_smooth(nx, ny, seed + 1)
    uy = wl.uy0 + amp_u * I.random_smooth(nx, ny, seed + 2)
    p = wl.p0 + amp_p * I.random_smooth(nx, ny, seed + 3)
    return I.Workload(wl.name, dict(wl.params), wl.phi0, ux, uy, p, wl.steps, dict(wl.meta))


def _walled_droplet():
    nx, ny = 520, 300
    phi = I.drop_field(nx, ny, 261.3, 148.6, 60.0, 4.0, periodic=False)
    z = np.zeros_like(phi)
    prm = I.base_params(nx, ny, wall_x=True, wall_y=True, rho1=1.0, rho2=1e-3, mu1=0.01,
                        mu2=1e-4, sigma=0.01, gy=-1e-6, rho_ref=1.0)
    return I.Workload("walled-droplet", prm, phi, z, z.copy(), z.copy(), 0)


CASES = {
    "capillary_128x512": lambda: _perturbed(I.capillary(nx=128, ny=512), 21),
    "rising_256x1024": lambda: _perturbed(I.rising_bubble(), 22),
    "droplet_520x300_walls": lambda: _perturbed(_walled_droplet(), 23),
}


def _fields(sim):
    f, g, u = (x.cpu() for x in sim.get_state())
    m = {k: v.cpu() for k, v in sim.moments().items()}
    return dict(f=f, g=g, u=u, phi=m["phi"], p=m["p"])


@pytest.mark.parametrize("case", list(CASES))
def test_walled_config_sizes_fp64(case):
    wl = CASES[case]()
    print(case, wl.params["nx"], wl.params["ny"], "walls", wl.params["wall_x"],
          wl.params["wall_y"], flush=True)
    st, prm = oracle_init(wl)
    sim = gpu_sim(wl)
    done = 0
    for n in (1, 5, 20):
        st = oracle.run(st, prm, n - done)
        sim.step(n - done)
        done = n
        got = _fields(sim)
        ref = dict(f=st.fs, g=st.gs, u=st.uo, phi=st.phi, p=st.p)
        errs = {k: relerr(got[k], ref[k]) for k in ref}
        bitwise = all(torch.equal(got[k], ref[k]) for k in ref)
        print(case, "step", n, {k: f"{e:.2e}" for k, e in errs.items()},
              "bitwise" if bitwise else "", flush=True)
        for k, e in errs.items():
            assert e <= RTOL64, (case, n, k, e)
    sim.close()


@pytest.mark.parametrize("case", list(CASES))
def test_walled_config_sizes_fp32_one_step(case):
    """One FP32 step from the oracle's state after 5 steps, against the oracle's
    FP64 step; errors over each field's maximum on the lattice."""
    wl = CASES[case]()
    st, prm = oracle_init(wl)
    st = oracle.run(st, prm, 5)
    sim = gpu_sim(wl, precision=1)
    sim.set_state(st.fs, st.gs, st.uo)
    sim.step(1)
    got = _fields(sim)
    sim.close()
    st = oracle.step_once(st, prm)
    ref = dict(f=st.fs, g=st.gs, u=st.uo, phi=st.phi, p=st.p)
    errs = {k: float((got[k] - ref[k]).abs().max()) / float(ref[k].abs().max()) for k in ref}
    print(case, "fp32", {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= RTOL32_STEP[k], (case, k, e)


def test_set_velocity_time_modulated_vortex():
    """Sec. 4.1: u(x, t) = u0(x) cos(pi t / T), prescribed before every step
    (here T = 100 steps, so that d_t u is far from zero), 128^2, 50 steps
    against the oracle's set_velocity, every 10 steps; a record right after
    a set_velocity is refused."""
    from paper_1812_02459_amd.binding import LBMError
    wl = I.vortex(n=128)
    T = 100.0
    st, prm = oracle_init(wl)
    sim = gpu_sim(wl)
    u0x, u0y = torch.tensor(wl.ux0), torch.tensor(wl.uy0)
    for n in range(1, 51):
        c = math.cos(math.pi * n / T)
        st = oracle.set_velocity(st, c * u0x, c * u0y)
        sim.set_velocity(c * u0x, c * u0y)
        st = oracle.step_once(st, prm)
        sim.step(1)
        if n % 10 == 0:
            f, _, u = sim.get_state()
            phi = sim.moments()["phi"]
            errs = dict(f=relerr(f, st.fs), u=relerr(u, st.uo), phi=relerr(phi, st.phi))
            print("modulated vortex step", n, {k: f"{e:.2e}" for k, e in errs.items()},
                  flush=True)
            for k, e in errs.items():
                assert e <= RTOL64, (n, k, e)
    sim.set_velocity(u0x, u0y)
    with pytest.raises(LBMError, match="call out of order"):
        sim.record(4, 2)
    # the held velocity: d_t u is zero again from the second step on
    st = oracle.set_velocity(st, u0x, u0y)
    st = oracle.run(st, prm, 3)
    sim.step(3)
    f, _, _ = sim.get_state()
    assert relerr(f, st.fs) <= RTOL64
    sim.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_state_is_reported(precision, bad):
    """A NaN or Inf injected into phi0 through lbm2p_init_fields spreads through
    the step; lbm2p_volume then returns ENONFINITE (the sums are not finite)."""
    from paper_1812_02459_amd.binding import lbm2p_volume, ENONFINITE, OK
    wl = I.droplet(n=64, seed=3, radii=(16,))
    phi0 = wl.phi0.copy()
    sim = gpu_sim(wl, precision=precision)
    code, _ = lbm2p_volume(sim.ctx)
    assert code == OK
    phi0[20, 31] = bad
    sim.init(phi0, wl.ux0, wl.uy0, wl.p0)
    sim.step(1)
    code, v = lbm2p_volume(sim.ctx)
    print("injected", bad, "precision", precision, "volume ->", code, v, flush=True)
    assert code == ENONFINITE
    assert not sim.volume()["finite"]
    sim.close()
