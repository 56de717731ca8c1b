"""Pins of the oracle's deforming-cell algebra.

exp(L tau) against scipy's matrix exponential (a library routine) and its
determinant; perpendicular widths against the closed form of a sheared
cube; the Lagrange-Gauss reduction against the defining properties of a
reduced basis of the same lattice; simple shear against textbook
Lees-Edwards flips; the Kraynik-Reinelt-aligned input lattice against its
integer self-map.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from paper_2512_13267_amd import inputs

GRADS = [
    (0.3, 0.2, -0.4),    # elliptic
    (0.4, 0.3, 0.2),     # hyperbolic
    (-0.5, 0.5, 0.5),    # hyperbolic
    (0.0, 0.1, 0.0),     # simple shear (parabolic, k = 0)
    (0.2, 0.4, -0.1),    # parabolic: a^2 + bc = 0
    (0.0, -0.3, 0.3),    # pure rotation
]


@pytest.mark.parametrize("abc", GRADS)
@pytest.mark.parametrize("tau", [0.005, 0.01, 1.0, 7.5])
def test_expL_matches_matrix_exponential(orc, abc, tau):
    L = inputs.planar_gradient(*abc)
    E = orc.expL(L, tau)
    ref = expm(L * tau)
    assert np.allclose(E, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert abs(np.linalg.det(E) - 1.0) < 1e-12 * np.abs(E).max() ** 2


def test_check_gradient(orc):
    assert orc.check_gradient(inputs.planar_gradient(0.1, 0.2, 0.3))
    bad = inputs.planar_gradient(0.1, 0.2, 0.3)
    bad[1, 1] = 0.2  # trace 0.3
    assert not orc.check_gradient(bad)
    bad = np.zeros((3, 3))
    bad[2, 0] = 0.1  # out of plane
    assert not orc.check_gradient(bad)
    bad = np.zeros((3, 3))
    bad[0, 1] = np.nan
    assert not orc.check_gradient(bad)


@pytest.mark.parametrize("t", [0.0, 0.3, -0.45, 1.7])
def test_widths_of_sheared_cube(orc, t):
    ell = 7.0
    h = np.array([[ell, t * ell, 0], [0, ell, 0], [0, 0, ell]])
    w = orc.widths(h)
    assert np.allclose(w, [ell / math.sqrt(1 + t * t), ell, ell], rtol=1e-14)


def test_reduce_cell_properties(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        B = rng.normal(size=(2, 2)) * rng.uniform(1, 20)
        B[:, 1] += rng.integers(-6, 7) * B[:, 0]  # skew the basis
        if abs(np.linalg.det(B)) < 1e-3:
            continue
        if np.linalg.det(B) < 0:
            B[:, 1] *= -1
        h = np.zeros((3, 3))
        h[:2, :2] = B
        h[2, 2] = 5.0
        hn, U, changed = orc.reduce_cell(h)
        assert round(np.linalg.det(U)) == 1
        assert np.allclose(h[:2, :2] @ U, hn[:2, :2], rtol=1e-10, atol=1e-10 * np.abs(B).max())
        b1, b2 = hn[:2, 0], hn[:2, 1]
        assert b1 @ b1 <= b2 @ b2 * (1 + 1e-12)
        assert abs(b1 @ b2) <= 0.5 * (b1 @ b1) * (1 + 1e-12)
        # reduced basis maximises the smaller width: it is the lattice's best
        assert min(orc.widths(hn)[:2]) >= inputs._lattice_min_width(B) * (1 - 1e-9)
        assert changed == (not np.array_equal(U, np.eye(2, dtype=np.int32)))


def test_simple_shear_flips_like_lees_edwards(orc):
    """Under u_x = rate*y the deformed cube is [[l, l*g], [0, l]] with
    strain g = rate*t; the reduced cell keeps the tilt in [-1/2, 1/2) * l,
    i.e. the Lees-Edwards image shift modulo one box length."""
    ell, rate, dt = 8.0, 0.7, 0.01
    L = inputs.shear_gradient(rate)
    E = orc.expL(L, dt)
    h = np.diag([ell, ell, ell])
    for n in range(1, 400):
        h = E @ h
        h, U, _ = orc.reduce_cell(h)
        g = rate * n * dt
        tilt = g - math.floor(g + 0.5)
        assert np.allclose(h[:2, 0], [ell, 0.0], atol=1e-9)
        assert abs(h[0, 1] - tilt * ell) < 1e-9 or abs(abs(h[0, 1] - tilt * ell) - ell) < 1e-9
        assert abs(h[1, 1] - ell) < 1e-9


@pytest.mark.parametrize("abc", [(0.4, 0.3, 0.2), (-0.45, 0.1, 0.35), (0.1, 0.5, 0.4)])
def test_kr_aligned_lattice_maps_onto_itself(abc):
    L = inputs.planar_gradient(*abc)
    h, kind = inputs.kr_cell(L, 9.0, 20.0)
    assert kind == "kr"
    k = math.sqrt(abc[0] ** 2 + abc[1] * abc[2])
    T = math.log((3 + math.sqrt(5)) / 2) / k
    P = h[:2, :2]
    M = np.linalg.inv(P) @ expm(L[:2, :2] * T) @ P
    assert np.allclose(M, np.round(M), atol=1e-8)
    assert abs(np.linalg.det(P) - 81.0) < 1e-9
    assert inputs._min_width_over(L[:2, :2], P, T, 65) >= 3.0
