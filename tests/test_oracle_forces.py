"""Pins of the oracle's pair search and forces (Eqs. F_DPD, conservative,
dissipative, random, fene_force).

* the cell-grid pair search finds exactly the brute-force O(N^2) x 27-image
  pair set, on cubic, sheared, reduced and Kraynik-Reinelt-aligned cells;
* total force vanishes (pairwise antisymmetry with theta_ij = theta_ji);
* conservative and FENE forces equal minus the finite-difference gradient of
  their potentials a rc/2 (1 - r/rc)^2 and -H R0^2/2 ln(1 - r^2/R0^2);
* an over-stretched bond raises the sticky BOND bit.
"""
import numpy as np
import pytest

from paper_2512_13267_amd import inputs


def _cells():
    out = [("cube", np.diag([4.3, 5.1, 4.6]))]
    sh = np.diag([5.0, 5.0, 4.0])
    sh[0, 1] = 2.2  # sheared, not reduced (tilt 0.44 l)
    out.append(("sheared", sh))
    L = inputs.planar_gradient(0.4, 0.3, 0.2)
    h, _ = inputs.kr_cell(L, 7.0, 20.0)
    out.append(("kr", h))
    g = np.array([[6.0, 1.7, 0.0], [-0.8, 5.5, 0.0], [0.0, 0.0, 3.4]])
    out.append(("general", g))
    return out


@pytest.mark.parametrize("name,h", _cells())
def test_cell_grid_finds_brute_force_pairs(orc, name, h):
    rng = np.random.default_rng(5)
    V = abs(np.linalg.det(h))
    N = int(3 * V)
    s = rng.random((N, 3))
    ij0, d0 = orc.pairs(s, h, 1.0, 0)
    ij1, d1 = orc.pairs(s, h, 1.0, 1)
    assert ij1 is not None
    assert len(ij0) > 0
    k0 = {(int(i), int(j)): d for (i, j), d in zip(ij0, d0)}
    k1 = {(int(i), int(j)): d for (i, j), d in zip(ij1, d1)}
    assert set(k0) == set(k1)
    for key in k0:
        assert np.allclose(k0[key], k1[key], atol=1e-12)
    # every kept pair is within the cutoff and the set matches a direct count
    r = np.linalg.norm(d0, axis=1)
    assert np.all((r > 0) & (r < 1.0))


def _state(name, h, seed=9, nch=None):
    rng = np.random.default_rng(seed)
    N = int(3 * abs(np.linalg.det(h)))
    nch = N // 50 if nch is None else nch
    s, c = inputs.random_box(rng, h, N, nch, 10)
    return s, c, nch


@pytest.mark.parametrize("name,h", _cells())
def test_forces_cell_grid_equal_brute_force_and_sum_to_zero(orc, name, h):
    p = inputs.default_params()
    s, c, nch = _state(name, h)
    L = inputs.planar_gradient(0.2, -0.3, 0.25)
    F0, W0, e0 = orc.forces(p, p["seed"], 10, 3, nch, s, c, h, L, 17, mode=0)
    F1, W1, e1 = orc.forces(p, p["seed"], 10, 3, nch, s, c, h, L, 17, mode=1)
    scale = np.abs(F0).max()
    assert np.allclose(F0, F1, atol=1e-12 * scale)
    assert np.allclose(W0, W1, atol=1e-11 * np.abs(W0).max())
    assert np.abs(F0.sum(axis=0)).max() < 1e-11 * scale
    assert e0 == e1 == 0


def _two_body(orc, p, r_vec, chain):
    h = np.diag([6.0, 6.0, 6.0])
    r0 = np.array([3.0, 3.0, 3.0])
    pos = np.stack([r0, r0 - r_vec])
    s = pos @ np.linalg.inv(h).T
    c = np.zeros((2, 3))
    F, W, err = orc.forces(p, 1, 2, 0, 1 if chain else 0, s, c, h, np.zeros((3, 3)), 0, mode=0)
    return F, W, err


def test_conservative_force_is_minus_gradient_of_potential(orc):
    p = inputs.default_params(gamma=0.0, sigma=0.0)
    a, rc = p["a"], p["rc"]

    def U(x):
        r = np.linalg.norm(x)
        return 0.5 * a * rc * (1 - r / rc) ** 2 if r < rc else 0.0

    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.normal(size=3)
        x *= rng.uniform(0.1, 0.95) / np.linalg.norm(x)
        F, _, _ = _two_body(orc, p, x, chain=False)
        eps = 1e-6
        g = np.array([(U(x + eps * e) - U(x - eps * e)) / (2 * eps) for e in np.eye(3)])
        assert np.allclose(F[0], -g, rtol=1e-7, atol=1e-8)
        assert np.allclose(F[0], -F[1], atol=1e-14)


def test_fene_force_is_minus_gradient_of_potential(orc):
    p = inputs.default_params(a=0.0, gamma=0.0, sigma=0.0)
    H, R0 = p["H"], p["R0"]

    def U(x):
        return -0.5 * H * R0 * R0 * np.log(1.0 - (x @ x) / (R0 * R0))

    rng = np.random.default_rng(2)
    for _ in range(20):
        x = rng.normal(size=3)
        x *= rng.uniform(0.2, 1.45) / np.linalg.norm(x)
        F, W, err = _two_body(orc, p, x, chain=True)
        eps = 1e-7
        g = np.array([(U(x + eps * e) - U(x - eps * e)) / (2 * eps) for e in np.eye(3)])
        assert np.allclose(F[0], -g, rtol=1e-7, atol=1e-7)
        assert err == 0
        # attractive: the force on bead 0 points toward bead 1
        assert F[0] @ x < 0


def test_overstretched_bond_sets_bond_flag(orc):
    p = inputs.default_params(a=0.0, gamma=0.0, sigma=0.0)
    x = np.array([1.01 * p["R0"], 0.0, 0.0])
    F, _, err = _two_body(orc, p, x, chain=True)
    assert err & orc.ERR_BOND
    # clamped denominator 0.01: |F| = H r / 0.01
    assert abs(np.linalg.norm(F[0]) - p["H"] * 1.01 * p["R0"] / 0.01) < 1e-9


def test_virial_is_symmetric_and_matches_pair_sum(orc):
    """The virial parts are sums of d (x) f over pairs with f parallel to d;
    the sum of the per-particle r_i (x) F_i over an isolated cluster (no
    periodic crossing) equals the pair virial."""
    p = inputs.default_params()
    h = np.diag([30.0, 30.0, 30.0])
    rng = np.random.default_rng(4)
    pos = 10.0 + rng.random((60, 3)) * 3.0  # a cluster far from the cell faces
    s = pos / 30.0
    c = rng.normal(size=(60, 3))
    F, W, _ = orc.forces(p, 5, 10, 0, 2, s, c, h, inputs.shear_gradient(0.3), 4, mode=0)
    Wt = W.sum(axis=0)
    full = pos.T @ F  # sum_i r_i F_i^T
    sym6 = np.array([full[0, 0], full[1, 1], full[2, 2], full[0, 1], full[0, 2], full[1, 2]])
    assert np.allclose(Wt, sym6, rtol=1e-10, atol=1e-10 * np.abs(full).max())
    assert np.allclose(full, full.T, atol=1e-10 * np.abs(full).max())
