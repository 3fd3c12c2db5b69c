"""Pins of the composed oracle step.

* TVD-RK3 driver: amplification 1 + z + z^2/2 + z^3/6 for a linear L (eq:TVD-3order);
* conservation on a periodic box: sum phi (streaming is a permutation, s0^f = 1 puts
  phi^{n+1} into the populations, the FD flux divergence telescopes) and sum p
  (filter mean-preserving, zero-mass source) stay constant;
* the step commutes with the x-mirror and with a 90-degree rotation (index bugs,
  sign errors and transposed operands break this);
* streaming equals an explicit permutation matrix built from index arithmetic,
  with half-way bounce-back at walls;
* the FD correction leaves the tanh profile (nearly) alone and its error shrinks
  at the stencil's order as the interface widens.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import step as S, ops
from oracle import lattice as L
from oracle import diagnostics as D
from paper_1812_02459_amd import inputs as I


def _t(a):
    return torch.tensor(a, dtype=torch.float64)


def test_rk3_amplification():
    phibar = _t(np.random.default_rng(0).uniform(-1, 1, (4, 5)))
    for z in (-0.9, -0.3, 0.2, 1.1):
        out = S.rk3(phibar, lambda q: z * q)
        assert torch.allclose(out, (1 + z + z * z / 2 + z ** 3 / 6) * phibar, atol=1e-15)


def _droplet_state(n=32, coupled=True, **kw):
    phi = I.drop_field(n, n, n / 2 + 0.3, n / 2 - 0.7, n / 4, 4.0)
    ux = 0.01 * I.random_smooth(n, n, 1)
    uy = 0.01 * I.random_smooth(n, n, 2)
    p = 1e-3 * I.random_smooth(n, n, 3)
    prm = oracle.Params(**I.base_params(n, n, coupled=coupled, rho1=1.0, rho2=1e-3,
                                        mu1=0.01, mu2=1e-4, sigma=0.01, **kw))
    return oracle.init_state(_t(phi), _t(ux), _t(uy), _t(p), prm), prm


@pytest.mark.parametrize("coupled", [True, False])
def test_conservation_periodic(coupled):
    st, prm = _droplet_state(coupled=coupled)
    s0 = float(st.fs.sum())
    p0 = float(st.gs.sum()) if coupled else 0.0
    for _ in range(20):
        st = oracle.step_once(st, prm)
        assert abs(float(st.fs.sum()) - s0) < 1e-12 * st.fs[0].numel()
        assert abs(D.total(st.phi) - s0) < 1e-12 * st.fs[0].numel()
        if coupled:
            assert abs(float(st.gs.sum()) - p0) < 1e-13 * st.fs[0].numel()


def _mirror_x(st):
    perm = [L.C.index((-cx, cy)) for (cx, cy) in L.C]

    def fld(a):
        return torch.roll(torch.flip(a, dims=(-1,)), shifts=1, dims=-1)
    fs = torch.stack([fld(st.fs[perm[i]]) for i in range(9)])
    gs = torch.stack([fld(st.gs[perm[i]]) for i in range(9)])
    uo = torch.stack([-fld(st.uo[0]), fld(st.uo[1])])
    return oracle.State(fs=fs, gs=gs, uo=uo)


def _rot90(st):
    # (x, y) -> (-y, x):  c_i -> R c_i, u -> R u
    perm = [L.C.index((cy, -cx)) for (cx, cy) in L.C]   # new_i = old_{R^-1 c_i}

    def fld(a):
        # new[y', x'] = old[y, x] with x' = -y, y' = x (periodic, node 0 fixed)
        b = a.transpose(-1, -2)                            # b[x, y] = a[y, x]
        return torch.roll(torch.flip(b, dims=(-1,)), shifts=1, dims=-1)
    fs = torch.stack([fld(st.fs[perm[i]]) for i in range(9)])
    gs = torch.stack([fld(st.gs[perm[i]]) for i in range(9)])
    uo = torch.stack([-fld(st.uo[1]), fld(st.uo[0])])
    return oracle.State(fs=fs, gs=gs, uo=uo)


@pytest.mark.parametrize("sym", [_mirror_x, _rot90])
def test_step_commutes_with_lattice_symmetries(sym):
    st, prm = _droplet_state(n=24)
    a = sym(oracle.run(st, prm, 2))
    b = oracle.run(sym(st), prm, 2)
    for x, y in ((a.fs, b.fs), (a.gs, b.gs), (a.uo, b.uo)):
        assert torch.allclose(x, y, atol=1e-14, rtol=0)


@pytest.mark.parametrize("walls", [(False, False), (False, True), (True, True)])
def test_streaming_permutation_matrix(walls):
    nx, ny = 6, 5
    prm = oracle.Params(nx=nx, ny=ny, wall_x=walls[0], wall_y=walls[1])
    fs = _t(np.random.default_rng(3).uniform(-1, 1, (9, ny, nx)))
    out = torch.stack(S.stream(fs, prm))
    # explicit matrix on the flattened (i, y, x) vector
    Nn = 9 * ny * nx
    P = np.zeros((Nn, Nn))
    for i, (cx, cy) in enumerate(L.C):
        for y in range(ny):
            for x in range(nx):
                sx, sy = x - cx, y - cy
                src_i = i
                out_x = not (0 <= sx < nx)
                out_y = not (0 <= sy < ny)
                if (walls[0] and out_x) or (walls[1] and out_y):
                    src_i, sx, sy = L.OPP[i], x, y        # half-way bounce-back
                P[(i * ny + y) * nx + x, (src_i * ny + sy % ny) * nx + sx % nx] = 1
    ref = (P @ fs.numpy().reshape(-1)).reshape(9, ny, nx)
    assert np.array_equal(out.numpy(), ref)


def _tanh_line(W, n=64):
    y = torch.arange(n, dtype=torch.float64)
    r = torch.minimum(y - n / 4, 3 * n / 4 - y)   # two interfaces on a periodic line
    return torch.tanh(2 * r / W)[:, None].expand(n, 8).contiguous()


def test_fd_correction_on_tanh_converges():
    errs = []
    for W in (4.0, 8.0, 16.0):
        n = int(16 * W)
        phi = _tanh_line(W, n)
        prm = oracle.Params(nx=8, ny=n, W=W, lam=0.05, M=0.0, sigma=0.0, eps=1e-12)
        L_ = S.fd_rhs(phi, prm)
        errs.append(float(L_.abs().max()))
    # J_phi(tanh) = 0 in the continuum (eps -> 0); the discrete L decays at least like W^-4
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12


def test_chemical_potential_of_tanh_converges():
    errs = []
    for W in (4.0, 8.0, 16.0):
        n = int(16 * W)
        phi = _tanh_line(W, n)
        prm = oracle.Params(nx=8, ny=n, W=W, sigma=1.0)
        mu = S.chem_pot(ops.ext(phi, 1), prm)
        scale = 3 * prm.sigma / W                     # size of each term of mu
        errs.append(float(mu.abs().max()) / scale)
    assert errs[0] < 0.1
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5   # O(W^-2)
