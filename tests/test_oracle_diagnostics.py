"""Pins of the oracle's rising-bubble diagnostics (eq:quantify-yc,
eq:quantify-uc): y_c and V_c, the means of the row index and of the vertical
velocity over the nodes with phi < 0, checked against what geometry and
linearity fix, and against brute force on small arrays."""

import math

import numpy as np
import torch

from oracle import diagnostics as D
from paper_1812_02459_amd import inputs as I


def _disk(nx, ny, xc, yc, R):
    return torch.tensor(I.drop_field(nx, ny, xc, yc, R, 4.0, inside=-1.0, periodic=False))


def test_centroid_of_a_symmetric_disk_is_its_centre_row():
    """A gas disk centred on a node row: the set phi < 0 is mirror-symmetric about
    that row, so y_c is the row exactly (sums of integers in float64)."""
    for (nx, ny, xc, yc, R) in [(64, 128, 32.0, 40.0, 12.0), (50, 90, 20.0, 61.0, 9.5)]:
        phi = _disk(nx, ny, xc, yc, R)
        area, y_c, v_c = D.bubble_stats(phi, torch.zeros_like(phi))
        assert y_c == yc
        assert v_c == 0.0
        # the area approximates the disk's: pi R^2 within the node-counting error
        assert abs(area - math.pi * R * R) < 2 * math.pi * R


def test_centroid_moves_with_the_bubble():
    """Moving the disk k rows up moves y_c by exactly k; the liquid side's mean row
    (a plausible sign mistake, phi > 0) is elsewhere."""
    nx, ny = 48, 160
    base = D.bubble_stats(_disk(nx, ny, 24.0, 50.0, 10.0), torch.zeros(ny, nx))
    for k in (1, 7, 33):
        moved = D.bubble_stats(_disk(nx, ny, 24.0, 50.0 + k, 10.0), torch.zeros(ny, nx))
        assert moved[0] == base[0] and moved[1] == base[1] + k
    phi = _disk(nx, ny, 24.0, 50.0, 10.0)
    liquid = D.bubble_stats(-phi, torch.zeros_like(phi))
    assert abs(liquid[1] - base[1]) > 20


def test_rise_velocity_is_the_mean_over_the_bubble():
    """V_c of a uniform v is v; of v = a y + b it is a y_c + b (linearity); the
    liquid's velocity does not enter."""
    nx, ny = 40, 100
    phi = _disk(nx, ny, 20.0, 37.0, 8.0)
    ys = torch.arange(ny, dtype=torch.float64)[:, None].expand(ny, nx)
    _, y_c, v_c = D.bubble_stats(phi, torch.full((ny, nx), 3.25e-3, dtype=torch.float64))
    assert abs(v_c - 3.25e-3) <= 1e-15
    a, b = 2e-5, -1e-3
    _, y_c, v_c = D.bubble_stats(phi, a * ys + b)
    assert abs(v_c - (a * y_c + b)) <= 1e-15
    v = torch.where(phi < 0, torch.tensor(1e-3, dtype=torch.float64), torch.tensor(5.0, dtype=torch.float64))
    assert abs(D.bubble_stats(phi, v)[2] - 1e-3) <= 1e-15


def test_brute_force_on_small_arrays():
    rng = np.random.default_rng(4)
    for _ in range(5):
        ny, nx = rng.integers(3, 8, size=2)
        phi = rng.uniform(-1, 1, size=(ny, nx))
        v = rng.normal(size=(ny, nx))
        cnt, sy, sv = 0, 0.0, 0.0
        for j in range(ny):
            for i in range(nx):
                if phi[j, i] < 0:
                    cnt += 1
                    sy += j
                    sv += v[j, i]
        area, y_c, v_c = D.bubble_stats(torch.tensor(phi), torch.tensor(v))
        assert area == cnt
        if cnt:
            assert abs(y_c - sy / cnt) <= 1e-12 and abs(v_c - sv / cnt) <= 1e-12
    area, y_c, v_c = D.bubble_stats(torch.ones(4, 4, dtype=torch.float64), torch.zeros(4, 4))
    assert area == 0 and math.isnan(y_c) and math.isnan(v_c)
