"""Pin of the adjoint's reference: torch autograd through one oracle step
(the derivative the GPU adjoint is compared with) against central differences
of the oracle itself, in FP64.

L = <cf, f*'> + <cg, g*'> + <cu, u~'> + <cphi, phi'> after one step of a 1000:1
droplet with walls in y and gravity, from a generic state (two steps after the
equilibrium start); derivatives with respect to sigma, M and a random
direction in the state (f*, g*, u~).  The step sizes keep the central
difference's truncation and rounding errors below the 1e-6 bar (sigma and M at
1e-3 relative agree to ~1e-9 here).
"""

import dataclasses

import torch

import oracle

from gpu_common import droplet_case, oracle_init


def _setup():
    wl = droplet_case(24, 20, seed=1, wall_y=True, gy=-1e-5)
    st, prm = oracle_init(wl)
    st = oracle.run(st, prm, 2)
    g = torch.Generator().manual_seed(0)
    r = lambda s: torch.randn(s, generator=g, dtype=torch.float64)
    cot = dict(f=r(st.fs.shape), g=r(st.gs.shape), u=r(st.uo.shape), phi=r(st.phi.shape))
    return st, prm, cot, r


def _loss(fs, gs, uo, prm, cot):
    s1 = oracle.step_once(oracle.State(fs=fs, gs=gs, uo=uo), prm)
    return ((s1.fs * cot["f"]).sum() + (s1.gs * cot["g"]).sum() + (s1.uo * cot["u"]).sum()
            + (s1.phi * cot["phi"]).sum())


def test_oracle_autograd_matches_central_differences():
    st, prm, cot, r = _setup()
    sig = torch.tensor(prm.sigma, dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(prm.M, dtype=torch.float64, requires_grad=True)
    fs = st.fs.clone().requires_grad_()
    gs = st.gs.clone().requires_grad_()
    uo = st.uo.clone().requires_grad_()
    L = _loss(fs, gs, uo, dataclasses.replace(prm, sigma=sig, M=Mt), cot)
    gfs, ggs, guo, gsig, gM = torch.autograd.grad(L, [fs, gs, uo, sig, Mt])
    vf, vg, vu = r(st.fs.shape), r(st.gs.shape), r(st.uo.shape)
    with torch.no_grad():
        def L_at(ds=0.0, dm=0.0, t=0.0):
            p = dataclasses.replace(prm, sigma=prm.sigma + ds, M=prm.M + dm)
            return float(_loss(st.fs + t * vf, st.gs + t * vg, st.uo + t * vu, p, cot))
        hs, hm, ht = 1e-3 * prm.sigma, 1e-3 * prm.M, 1e-6
        fd_s = (L_at(ds=hs) - L_at(ds=-hs)) / (2 * hs)
        fd_m = (L_at(dm=hm) - L_at(dm=-hm)) / (2 * hm)
        fd_t = (L_at(t=ht) - L_at(t=-ht)) / (2 * ht)
    ad_t = float((gfs * vf).sum() + (ggs * vg).sum() + (guo * vu).sum())
    for name, ad, fd in (("sigma", float(gsig), fd_s), ("M", float(gM), fd_m), ("state", ad_t, fd_t)):
        assert abs(ad - fd) <= 1e-6 * abs(fd), (name, ad, fd)


def test_planted_sign_error_in_a_force_term_is_caught():
    """The derivative changes measurably when the sigma-dependent part of the
    oracle's force enters with the wrong sign (a planted mistake, on the CPU):
    the adjoint tests built on this reference would catch such a mistake."""
    from oracle import step as S
    st, prm, cot, r = _setup()
    orig = S.forces
    sig = torch.tensor(prm.sigma, dtype=torch.float64, requires_grad=True)
    fs = st.fs.clone()
    L = _loss(fs, st.gs, st.uo, dataclasses.replace(prm, sigma=sig), cot)
    (g_true,) = torch.autograd.grad(L, [sig])
    # planted mistake: the surface-force contribution enters with the wrong sign
    S.forces = lambda phi, p, ux, uy, prm_, g=None: _flip_fs(orig, phi, p, ux, uy, prm_, g=g)
    try:
        sig2 = torch.tensor(prm.sigma, dtype=torch.float64, requires_grad=True)
        L2 = _loss(fs, st.gs, st.uo, dataclasses.replace(prm, sigma=sig2), cot)
        (g_bad,) = torch.autograd.grad(L2, [sig2])
    finally:
        S.forces = orig
    assert abs(float(g_bad) - float(g_true)) > 1e-6 * abs(float(g_true))


def _flip_fs(orig, phi, p, ux, uy, prm, g=None):
    """forces() with the surface force's sign reversed (planted mistake)."""
    d = dict(orig(phi, p, ux, uy, prm, g=g))
    z = dataclasses.replace(prm, sigma=0.0 * prm.sigma)
    d0 = orig(phi, p, ux, uy, z, g=g)
    # F(sigma) - F(0) is the sigma-dependent part (F_s plus J's mu terms)
    d["Fx"] = d0["Fx"] - (d["Fx"] - d0["Fx"])
    d["Fy"] = d0["Fy"] - (d["Fy"] - d0["Fy"])
    return d
