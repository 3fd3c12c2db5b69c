"""Adjoint (reverse mode) of the HIP library, through the C-ABI, against torch
autograd of the CPU oracle (FP64, same seeded inputs).

The oracle is plain torch, so autograd through its step is the exact
derivative of the oracle's arithmetic (its square root has a hand-written
derivative 1/(2 sqrt), and torch's clamp passes the derivative for
-1 <= phi <= 1, ends included, as the library does).  The GPU adjoint sums its
terms in another order, so the bar is a relative error (max norm over max norm,
or relative for a scalar) of 1e-10, not bitwise.
"""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1812_02459_amd import inputs as I

from gpu_common import relerr, oracle_init, gpu_sim, droplet_case

pytestmark = pytest.mark.gpu

RTOL_ADJ = 1e-10


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


def _scalar_err(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _cotangents(shape_f, shape_u, ny, nx, coupled, seed):
    g = torch.Generator().manual_seed(seed)
    r = lambda *s: torch.randn(*s, generator=g, dtype=torch.float64)
    return dict(f=r(*shape_f), g=r(*shape_f) if coupled else None, u=r(*shape_u) if coupled else None,
                phi=r(ny, nx))


def _oracle_step_vjp(st, prm, cot):
    """Autograd of one oracle step: gradients of
    L = <cf, f*'> + <cg, g*'> + <cu, u~'> + <cphi, phi'> with respect to the
    state (f*, g*, u~) and to sigma, M."""
    sig = torch.tensor(prm.sigma, dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(prm.M, dtype=torch.float64, requires_grad=True)
    fs = st.fs.clone().requires_grad_()
    gs = st.gs.clone().requires_grad_() if st.gs is not None else None
    uo = st.uo.clone().requires_grad_()
    p2 = dataclasses.replace(prm, sigma=sig, M=Mt)
    s1 = oracle.step_once(oracle.State(fs=fs, gs=gs, uo=uo), p2)
    L = (s1.fs * cot["f"]).sum() + (s1.phi * cot["phi"]).sum()
    wrt = [fs, uo, sig, Mt]
    if prm.coupled:
        L = L + (s1.gs * cot["g"]).sum() + (s1.uo * cot["u"]).sum()
        wrt.append(gs)
    gr = torch.autograd.grad(L, wrt, allow_unused=True)
    out = dict(f0=gr[0], sigma=float(gr[2]), M=float(gr[3]))
    if prm.coupled:
        out["u0"] = gr[1]
        out["g0"] = gr[4]
    return out


def _check(label, got, ref, keys):
    errs = {}
    for k in keys:
        if k in ("sigma", "M"):
            errs[k] = _scalar_err(got[k], ref[k])
        else:
            errs[k] = relerr(got[k], ref[k])
    print(label, {k: f"{v:.2e}" for k, v in errs.items()},
          f"sigma {got['sigma']:.6e} / {ref['sigma']:.6e}", f"M {got['M']:.6e} / {ref['M']:.6e}",
          flush=True)
    for k, v in errs.items():
        assert v <= RTOL_ADJ, (label, k, v)


ONE_STEP_CASES = [
    dict(),
    dict(wall_y=True, gy=-1e-5),
    dict(wall_x=True, wall_y=True, K=3, filter_n=7, gx=2e-6, gy=-1e-5),
    dict(filter_n=0, K=1),
    dict(original_ch=True, filter_n=5),
    dict(wall_x=True, filter_n=9, filter_a=0.3, K=4),
]


@pytest.mark.parametrize("kw", ONE_STEP_CASES)
def test_one_step_vjp_coupled(kw):
    """One reversed step from a generic state (two oracle steps after init),
    every seed and every output checked."""
    wl = droplet_case(24, 20, seed=3, **kw)
    st, prm = oracle_init(wl)
    st = oracle.run(st, prm, 2)
    cot = _cotangents(st.fs.shape, st.uo.shape, 20, 24, True, seed=11)
    ref = _oracle_step_vjp(st, prm, cot)
    sim = gpu_sim(wl)
    sim.set_state(st.fs, st.gs, st.uo)
    sim.record(1, 1)
    got = sim.adjoint(dL_dphi=cot["phi"], dL_df=cot["f"], dL_dg=cot["g"], dL_du=cot["u"],
                      want_state=True)
    _check(f"one step {kw}", got, ref, ("f0", "g0", "u0", "sigma", "M"))


def test_one_step_vjp_ch_only():
    wl = I.vortex(n=40)
    st, prm = oracle_init(wl)
    st = oracle.run(st, prm, 3)
    cot = _cotangents(st.fs.shape, st.uo.shape, 40, 40, False, seed=12)
    ref = _oracle_step_vjp(st, prm, cot)
    sim = gpu_sim(wl)
    sim.set_state(st.fs, None, st.uo)
    sim.record(1, 1)
    got = sim.adjoint(dL_dphi=cot["phi"], dL_df=cot["f"], want_state=True)
    _check("one step CH-only", got, ref, ("f0", "sigma", "M"))


def _oracle_run_grad(wl, nsteps, cphi):
    """Autograd of phi after nsteps steps from the equilibrium initial state:
    gradients of <cphi, phi_T> with respect to phi0, sigma, M."""
    p = dict(wl.params)
    prm = oracle.Params(**p)
    sig = torch.tensor(prm.sigma, dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(prm.M, dtype=torch.float64, requires_grad=True)
    phi0 = _t(wl.phi0).requires_grad_()
    p2 = dataclasses.replace(prm, sigma=sig, M=Mt)
    st = oracle.init_state(phi0, _t(wl.ux0), _t(wl.uy0), _t(wl.p0), p2)
    st = oracle.run(st, p2, nsteps)
    L = (st.phi * cphi).sum()
    g = torch.autograd.grad(L, [phi0, sig, Mt])
    return dict(phi0=g[0], sigma=float(g[1]), M=float(g[2]))


@pytest.mark.parametrize("case", ["walls", "periodic", "ch_only"])
def test_checkpointed_run_gradient(case):
    """Several segments (7 steps, a checkpoint every 3), the loss on the last
    phi, gradients down to phi0 through the equilibrium initial state."""
    if case == "walls":
        wl = droplet_case(32, 24, seed=5, wall_x=True, wall_y=True, gy=-1e-5)
    elif case == "periodic":
        wl = droplet_case(28, 32, seed=6, K=3)
    else:
        wl = I.vortex(n=32)
    ny, nx = wl.phi0.shape
    cphi = torch.randn(ny, nx, generator=torch.Generator().manual_seed(13), dtype=torch.float64)
    ref = _oracle_run_grad(wl, 7, cphi)
    sim = gpu_sim(wl)
    sim.record(7, 3)
    got = sim.adjoint(dL_dphi=cphi, want_phi0=True)
    _check(f"7 steps / 3 ({case})", got, ref, ("phi0", "sigma", "M"))
    # the context is back at the recorded final state
    st, prm = oracle_init(wl)
    st = oracle.run(st, prm, 7)
    assert relerr(sim.moments()["phi"], st.phi) <= 1e-12


def test_zero_steps_and_state_errors():
    from paper_1812_02459_amd.binding import LBMError
    wl = droplet_case(24, 20, seed=7)
    sim = gpu_sim(wl)
    with pytest.raises(LBMError, match="call out of order"):
        sim.adjoint(dL_dphi=np.ones((20, 24)))            # no record yet
    sim.record(0, 4)
    cphi = torch.randn(20, 24, generator=torch.Generator().manual_seed(14), dtype=torch.float64)
    got = sim.adjoint(dL_dphi=cphi, want_phi0=True)
    assert torch.equal(got["phi0"].cpu(), cphi)           # phi_T = phi0
    assert got["sigma"] == 0.0 and got["M"] == 0.0
    sim.record(2, 1)
    sim.step(1)                                           # the record is stale now
    with pytest.raises(LBMError, match="call out of order"):
        sim.adjoint(dL_dphi=cphi)
    sim.record(1, 1)                                      # not from the initial state
    with pytest.raises(LBMError, match="call out of order"):
        sim.adjoint(dL_dphi=cphi, want_phi0=True)


def test_autograd_function_small_rising_bubble():
    """The torch.autograd.Function (sigma, M, phi0) -> phi_T with the library's
    adjoint as backward, on a reduced closed-box rising bubble (64 x 256, R = 8,
    120 steps), against oracle autograd of L = mean((phi_T - phi*)^2)."""
    from paper_1812_02459_amd.binding import phase_field_run
    wl = I.rising_bubble(nx=64, ny=256, R=8.0, xc=32.0, yc=48.0, U_g=2e-3)
    nsteps = 120
    rng = np.random.default_rng(0)
    target = _t(np.tanh(rng.normal(size=wl.phi0.shape)))
    prm = dict(wl.params)
    sig = torch.tensor(prm["sigma"], dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(prm["M"], dtype=torch.float64, requires_grad=True)
    phi0 = _t(wl.phi0).cuda().requires_grad_()
    phiT = phase_field_run(sig, Mt, phi0, prm, nsteps, ckpt_every=32)
    L = ((phiT - target.cuda()) ** 2).mean()
    L.backward()
    got = dict(phi0=phi0.grad, sigma=float(sig.grad), M=float(Mt.grad))
    cphi = 2.0 * (phiT.detach().cpu() - target) / target.numel()
    ref = _oracle_run_grad(wl, nsteps, cphi)
    _check("autograd.Function rising bubble 64x256", got, ref, ("phi0", "sigma", "M"))
