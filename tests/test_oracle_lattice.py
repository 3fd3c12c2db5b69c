"""Pins of the oracle's lattice constants (D2Q9, MRT matrix, filter table).

The MRT rows are checked against the polynomial moment basis they stand for
(1, e = 3|c|^2 - 4, eps = (9|c|^4 - 21|c|^2)/2 + 4, j, q = (3|c|^2 - 5) c, p_xx,
p_xy); the weights against the isotropy conditions of a second-order lattice.
"""

import os
from fractions import Fraction

import numpy as np

from oracle import lattice as L

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append(line.split())
    return rows


def test_velocities_and_opposites():
    assert L.C[0] == (0, 0)
    assert set(L.C[1:5]) == {(1, 0), (0, 1), (-1, 0), (0, -1)}
    assert set(L.C[5:]) == {(1, 1), (-1, 1), (-1, -1), (1, -1)}
    for i in range(9):
        j = L.OPP[i]
        assert L.C[j] == (-L.C[i][0], -L.C[i][1])


def test_weights_isotropy():
    w = np.array(L.W)
    c = np.array(L.C, dtype=float)
    assert abs(w.sum() - 1.0) < 1e-15
    # sum w c_a c_b = c_s^2 delta_ab with c_s^2 = 1/3
    T2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(T2, np.eye(2) / 3, atol=1e-15)
    # fourth-order isotropy: sum w c_a c_b c_c c_d = c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(2)
    ref = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(T4, ref, atol=1e-15)
    # odd moments vanish
    assert np.allclose(np.einsum("i,ia->a", w, c), 0)


def test_mrt_matrix_matches_golden_and_polynomial_basis():
    gold = [[int(v) for v in r] for r in _read_rows("d2q9_mrt_matrix.txt")]
    assert [list(r) for r in L.M] == gold
    basis = []
    for (cx, cy) in L.C:
        c2 = cx * cx + cy * cy
        basis.append([1, 3 * c2 - 4, Fraction(9 * c2 * c2 - 21 * c2, 2) + 4, cx,
                      (3 * c2 - 5) * cx, cy, (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy])
    B = np.array(basis, dtype=float).T
    assert np.array_equal(B, np.array(L.M, dtype=float))


def test_mrt_orthogonality_and_inverse():
    M = np.array(L.M, dtype=float)
    MMt = M @ M.T
    assert np.array_equal(MMt, np.diag(np.diag(MMt)))
    assert tuple(np.diag(MMt)) == (9, 36, 36, 6, 12, 6, 12, 4, 4)
    Minv = M.T @ np.diag(L.MM_DIAG_INV)
    assert np.allclose(Minv @ M, np.eye(9), atol=1e-15)
    assert np.allclose(Minv, np.linalg.inv(M), atol=1e-15)


def test_filter_table_matches_golden_and_normalisation():
    for r in _read_rows("app_b_selective_filter.txt"):
        n = int(r[0].split("-")[1])
        vals = [float(Fraction(v)) if "/" in v else float(v) for v in r[1:]]
        assert np.allclose(L.FILTER_D[n], vals, rtol=0, atol=0)
        d = np.array(vals)
        m = np.arange(len(d))
        D0 = d[0] + 2 * d[1:].sum()                         # D(k=0)
        Dpi = d[0] + 2 * (d[1:] * np.cos(np.pi * m[1:])).sum()  # D(k=pi)
        assert abs(D0) < 1e-11
        assert abs(Dpi - 1.0) < 1e-11
