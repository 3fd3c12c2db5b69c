"""Parity at full size: the 4096^2 bubble ensemble in the launch configuration
bench.py times, checked on sampled windows the oracle can compute.

One step has a finite domain of dependence: a node's post-collision state at
n+1 depends on the state at n within 25 nodes (gather 1, three FD stages 5
each, K = 2 velocity sweeps and the filter 5 + 2 + 1, collide 2).  The oracle
advances an 80x80 periodic window cut from the GPU state at step n; the centre
16x16 (32 nodes from every window edge) must equal the GPU state at n+1.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1812_02459_amd import inputs as I

from gpu_common import RTOL64, relerr

pytestmark = pytest.mark.gpu

HALO = 32
CORE = 16


def _window(a, cx, cy):
    """(..., ny, nx) -> (..., CORE + 2 HALO, same) window starting at (cx - HALO, cy - HALO),
    wrapping periodically."""
    a = torch.roll(a, shifts=(-(cy - HALO), -(cx - HALO)), dims=(-2, -1))
    n = CORE + 2 * HALO
    return a[..., :n, :n]


def test_bubble_ensemble_sampled_windows():
    from paper_1812_02459_amd.binding import Sim
    wl = I.bubble_ensemble(n=4096, nb=200, seed=0)
    sim = Sim(wl.params, precision=0)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    sim.step(30)
    f, g, u = (x.cpu() for x in sim.get_state())
    sim.step(1)
    f1, g1, u1 = (x.cpu() for x in sim.get_state())
    m1 = {k: v.cpu() for k, v in sim.moments().items()}
    rng = np.random.default_rng(1)
    # windows on bubble interfaces, one across the periodic corner, random ones
    centres = []
    for (bx, by, R) in wl.meta["bubbles"][:4]:
        centres.append((int(bx + R) % 4096, int(by) % 4096))
    centres.append((4090, 4093))
    centres += [tuple(int(v) for v in rng.integers(0, 4096, 2)) for _ in range(3)]
    p = dict(wl.params)
    p["nx"] = p["ny"] = CORE + 2 * HALO
    prm = oracle.Params(**p)
    for (cx, cy) in centres:
        st = oracle.State(fs=_window(f, cx, cy), gs=_window(g, cx, cy), uo=_window(u, cx, cy))
        st = oracle.step_once(st, prm)
        c = slice(HALO, HALO + CORE)
        pairs = {"f": (_window(f1, cx, cy)[:, c, c], st.fs[:, c, c]),
                 "g": (_window(g1, cx, cy)[:, c, c], st.gs[:, c, c]),
                 "u": (_window(u1, cx, cy)[:, c, c], st.uo[:, c, c]),
                 "phi": (_window(m1["phi"], cx, cy)[c, c], st.phi[c, c]),
                 "p": (_window(m1["p"], cx, cy)[c, c], st.p[c, c])}
        for k, (a, b) in pairs.items():
            e = relerr(a, b)
            print((cx, cy), k, f"{e:.2e}", "bitwise" if torch.equal(a, b) else "", flush=True)
            assert e <= RTOL64, ((cx, cy), k, e)
