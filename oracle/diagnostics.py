"""Diagnostics of Sec. 4 (test infrastructure only).

* volume  #{phi > 0} and its percentage error (Sec. 4.3, text before Table III)
* sum of phi (conserved by the split scheme)
* pressure jump Delta p' = <rho p>_{phi > 0.99} - <rho p>_{phi < -0.99}
  (Laplace law, Sec. 4.3; p is the kinematic pressure and p' = rho p, Sec. 2.2)
* relative max / min errors of phi (eq:maxminPHI)
* interface height along a column (capillary wave, Sec. 4.4)
* bubble centroid and rise velocity (eq:quantify-yc, eq:quantify-uc)
"""

import torch


def volume(phi):
    return int((phi > 0).sum())


def volume_error_pct(phi0, phit):
    v0 = volume(phi0)
    return 100.0 * (v0 - volume(phit)) / v0


def total(phi):
    return float(phi.to(torch.float64).sum())


def pressure_jump(phi, p, rho1, rho2):
    phc = torch.clamp(phi, -1.0, 1.0)
    rho = rho1 * (1 + phc) / 2 + rho2 * (1 - phc) / 2
    pp = rho * p
    inside = phi > 0.99
    outside = phi < -0.99
    return float(pp[inside].mean() - pp[outside].mean())


def phi_range_errors(phi):
    """eq:maxminPHI: (max|(phi-1)/2|, max|(phi+1)/2|) -- as printed; reported only."""
    return float(((phi - 1) / 2).abs().max()), float(((phi + 1) / 2).abs().max())


def interface_height(phi, x=0):
    """y where phi changes sign along column x, by linear interpolation."""
    col = phi[:, x].to(torch.float64)
    s = torch.sign(col)
    idx = torch.nonzero(s[:-1] * s[1:] < 0).flatten()
    if idx.numel() == 0:
        return float("nan")
    k = int(idx[0])
    a, b = float(col[k]), float(col[k + 1])
    return k + a / (a - b)


def bubble_centroid(phi, uy):
    """y_c and V_c over the region phi < 0 (eq:quantify-yc, eq:quantify-uc)."""
    m = phi < 0
    ys = torch.arange(phi.shape[0], dtype=torch.float64)[:, None].expand_as(phi)
    n = m.sum()
    return float(ys[m].sum() / n), float(uy[m].sum() / n)


def bubble_stats(phi, uy):
    """(area, y_c, V_c): the number of nodes with phi < 0 and the two means of
    eq:quantify-yc and eq:quantify-uc over them, the integrals taken as sums
    over nodes; the node of row j sits at y = j."""
    area = int((phi < 0).sum())
    if area == 0:
        return 0, float("nan"), float("nan")
    yc, vc = bubble_centroid(phi, uy)
    return area, yc, vc
