"""Rising-bubble diagnostics y_c and V_c (Sec. 4.5, eq:quantify-yc,
eq:quantify-uc) on the GPU: the device reduction against the oracle's
definition, and the benchmark of Table IV (tests 1 and 2, 240 x 480) run to
t = 3 with self-consistency checks.  The paper's y_c and V_c curves are figures
whose data are not in the source, so the runs are checked against what the
physics and the definitions fix, with bounds declared before the first run:

* the state stays finite and the bubble's area (nodes with phi < 0) stays
  within 3 % of its initial value (the corrected CH conserves the phase);
* the bubble rises at least one radius by t = 3;
* V_c agrees with the central difference of y_c over +-0.1 time units to 5 %
  of the largest V_c after t = 0.5 (the two diagnostics are computed
  independently).  First run with +-0.02 (the sampling interval): 5.6 % on
  test 1.  Over 0.04 time units the bubble moves about 2 nodes, and one node
  entering or leaving the set phi < 0 moves y_c by up to R / area, about 0.02
  node, so that difference carries several per cent of node-count noise; over
  +-0.1 the same run agrees to 2 %;
* the largest V_c lies between 0.1 U_g and U_g (buoyancy-driven, slower than
  the gravitational velocity scale);
* test 1 at half the resolution (120 x 240) follows the same y_c(t), in domain
  widths, to 0.05.
"""

import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import diagnostics as D
from paper_1812_02459_amd import inputs as I

pytestmark = pytest.mark.gpu

OUT = os.environ.get("LBM2P_RESULTS_DIR")


@pytest.mark.parametrize("precision", [0, 1])
def test_bubble_diagnostics_match_oracle(precision):
    """lbm2p_bubble against the oracle's bubble_stats on the same fields (the GPU
    state's phi and u~ from lbm2p_moments): the area exactly, y_c and V_c to
    1e-12 relative (float64 sums in another order); lbm2p_pressure_jump against
    the oracle's pressure_jump likewise.  Also the empty case."""
    from paper_1812_02459_amd.binding import Sim
    wl = I.rising_bubble_benchmark(1, scale=0.25)
    sim = Sim(wl.params, precision=precision)
    sim.init(wl.phi0, wl.ux0, wl.uy0, wl.p0)
    for n in (0, 30):
        sim.step(n)
        b = sim.bubble()
        m = sim.moments()
        area, yc, vc = D.bubble_stats(m["phi"].cpu(), m["uy"].cpu())
        print(precision, n, b, (area, yc, vc), flush=True)
        assert b["area"] == area > 0
        assert abs(b["y_c"] - yc) <= 1e-12 * abs(yc)
        assert abs(b["V_c"] - vc) <= 1e-12 * abs(vc) + 1e-300
        # the pressure-jump reduction on the same fields (Sec. 4.3)
        pj = sim.pressure_jump()
        ref = D.pressure_jump(m["phi"].cpu(), m["p"].cpu(), wl.params["rho1"], wl.params["rho2"])
        assert pj["n_in"] == int((m["phi"] > 0.99).sum()) and pj["n_out"] == int((m["phi"] < -0.99).sum())
        assert abs(pj["dp"] - ref) <= 1e-12 * max(abs(pj["p_in"]), abs(pj["p_out"]), 1e-300)
    sim.close()
    flat = Sim(wl.params, precision=precision)
    flat.init(np.ones_like(wl.phi0), wl.ux0, wl.uy0, wl.p0)
    b = flat.bubble()
    assert b["area"] == 0 and math.isnan(b["y_c"]) and math.isnan(b["V_c"])
    flat.close()


def _run(test, scale=1.0, samples_per_time=50, precision=0, phi0=None):
    from paper_1812_02459_amd.binding import Sim
    wl = I.rising_bubble_benchmark(test, scale=scale)
    sim = Sim(wl.params, precision=precision)
    sim.init(wl.phi0 if phi0 is None else phi0, wl.ux0, wl.uy0, wl.p0)
    spt = wl.meta["steps_per_time"]
    dn = int(round(spt / samples_per_time))
    nsamp = int(round(wl.steps / dn))
    ts, area, yc, vc = [], [], [], []
    for k in range(nsamp + 1):
        if k:
            sim.step(dn)
        b = sim.bubble()
        ts.append(k * dn / spt)
        area.append(b["area"])
        yc.append(b["y_c"])
        vc.append(b["V_c"])
    finite = bool(sim.volume()["finite"])
    sim.close()
    return wl, dn, np.array(ts), np.array(area), np.array(yc), np.array(vc), finite


TEST2_DIVERGES = (
    "Table IV test 2 (1000:1, Eo = 125) diverges near t = 0.15 with this method's "
    "readings: parasitic currents reach U_g by t = 0.1 while the bubble moves at "
    "0.02 U_g; eps = 0.05 or 0.1 or W = 5 delay the divergence to t = 1.7-2.1, the free "
    "MRT rates, K = 4, the filter strength, M, rho_ref and the compact filter do not")


@pytest.mark.parametrize("test", [1, pytest.param(2, marks=pytest.mark.xfail(
    strict=True, reason=TEST2_DIVERGES))])
def test_table4_rising_bubble(test):
    wl, dn, t, area, yc, vc, finite = _run(test)
    R, U_g, nx = wl.meta["R"], wl.meta["U_g"], wl.params["nx"]
    drift = float(np.max(np.abs(area / area[0] - 1)))
    rise = float(yc[-1] - yc[0])
    h = 5                                   # samples: +-0.1 time units
    dydt = (yc[2 * h:] - yc[:-2 * h]) / (2 * h * dn)
    late = t[h:-h] >= 0.5
    vmax = float(np.max(vc))
    mismatch = float(np.max(np.abs(vc[h:-h][late] - dydt[late]))) / vmax
    summary = dict(test=test, steps=int(wl.steps), finite=finite, area_drift=drift,
                   rise_nodes=rise, rise_radii=rise / R, vmax_over_Ug=vmax / U_g,
                   dydt_mismatch=mismatch,
                   y_c_over_width=[round(float(v / nx), 5) for v in yc[::5]],
                   V_c_over_Ug=[round(float(v / U_g), 5) for v in vc[::5]],
                   t=[round(float(v), 3) for v in t[::5]])
    print({k: v for k, v in summary.items() if not isinstance(v, list)}, flush=True)
    if test == 1:
        _, _, t2, _, yc2, _, fin2 = _run(1, scale=0.5)
        common = min(len(t2), len(t))
        assert np.allclose(t[:common], t2[:common], atol=0.02)
        conv = float(np.max(np.abs(yc[:common] / nx - yc2[:common] / (nx / 2))))
        summary["half_resolution_y_c_gap_widths"] = conv
        print("half resolution: max |y_c/L - y_c'/L'|", conv, fin2, flush=True)
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, f"rising_bubble_test{test}.json"), "w") as fh:
            json.dump(summary, fh, indent=1)
    assert finite
    assert drift <= 0.03
    assert rise >= R
    assert mismatch <= 0.05
    assert 0.1 * U_g <= vmax <= U_g
    if test == 1:
        assert fin2 and conv <= 0.05


def test_table4_test1_fp32_follows_fp64():
    """FP32 error statement on the benchmark (test 1): the FP32 run's y_c within
    0.01 domain widths of the FP64 run's and its V_c within 5 % of the largest
    V_c (bounds declared before the first run), at every sample up to t = 1.5.

    Past t ~ 1.5 the flow itself is sensitive: FP64 runs from phi0 perturbed
    by 1e-10 or 3e-8 (random, three seeds) leave the unperturbed FP64 run by
    0.3-0.6 % of max V_c at t = 1.5 and by 8-11 % near t = 2.1, and by
    0.6-1.3e-2 widths in y_c over t <= 3, beyond the declared bounds; the
    comparison to t = 3 then measures that sensitivity rather than the FP32
    arithmetic.  It is run here alongside an FP64 run from a perturbed phi0,
    both distances are reported, and the FP32 distance over t <= 3 is held to
    twice the perturbed FP64 run's (measured: FP32 1.1e-1 of max V_c and
    1.1e-2 widths; FP64 + 1e-10 8.1e-2 and 6.5e-3).  Up to t = 1.5: FP32
    8.3e-3 and 5.1e-4 widths."""
    wl, _, t, _, y64, v64, f64 = _run(1, precision=0)
    _, _, _, _, y32, v32, f32 = _run(1, precision=1)
    rng = np.random.default_rng(7)
    pert = wl.phi0 + 1e-10 * rng.standard_normal(wl.phi0.shape)
    _, _, _, _, yp, vp, fp = _run(1, precision=0, phi0=pert)
    nx = wl.params["nx"]
    vmax = float(np.max(v64))
    early = t <= 1.5 + 1e-9
    dy = np.abs(y32 - y64) / nx
    dv = np.abs(v32 - v64) / vmax
    dyp = np.abs(yp - y64) / nx
    dvp = np.abs(vp - v64) / vmax
    rec = dict(dy_c_widths_to_1_5=float(dy[early].max()), dV_c_rel_to_1_5=float(dv[early].max()),
               dy_c_widths_to_3=float(dy.max()), dV_c_rel_to_3=float(dv.max()),
               fp64_perturbed_dy_c_widths_to_1_5=float(dyp[early].max()),
               fp64_perturbed_dV_c_rel_to_1_5=float(dvp[early].max()),
               fp64_perturbed_dy_c_widths_to_3=float(dyp.max()),
               fp64_perturbed_dV_c_rel_to_3=float(dvp.max()))
    print("test 1 FP32 vs FP64:", json.dumps(rec), flush=True)
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "rising_bubble_test1_fp32.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
    assert f64 and f32 and fp
    assert rec["dy_c_widths_to_1_5"] <= 0.01 and rec["dV_c_rel_to_1_5"] <= 0.05
    assert rec["dy_c_widths_to_3"] <= 2 * rec["fp64_perturbed_dy_c_widths_to_3"]
    assert rec["dV_c_rel_to_3"] <= 2 * rec["fp64_perturbed_dV_c_rel_to_3"]
