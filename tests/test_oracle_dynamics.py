"""Pins of the oracle's time stepping and stress (Eq. motion integrated by
velocity-Verlet; Eqs. IKtotal, kinetic_stress, potential_stress).

* free particles under simple shear travel in straight lines in the lab
  frame through every Lees-Edwards flip (exact for the scheme when L^2 = 0);
* with the thermostat off (gamma = sigma = 0, L = 0) velocity-Verlet keeps
  the total energy to O(dt^2) with no drift;
* equilibrium kinetic temperature equals kBT (fluctuation-dissipation with
  the discrete random force scaled by 1/sqrt(dt));
* with a = 0 the dissipative shear stress equals the closed form
  eta_D * rate, eta_D = 2 pi gamma rho^2 rc^5 / 1575 (pair density rho^2/2,
  g(r) = 1, angular mean of e_x^2 e_y^2 = 1/15, int r^4 (1-r)^2 dr = 1/105);
* the Newtonian solvent limit (no chains, a = 25): the shear stress is
  linear in the rate, sigma_xy / rate agrees over rates 0.05, 0.1, 0.2
  within two combined standard errors, and both normal-stress differences
  vanish within two standard errors;
* pure rotation gives no deviatoric stress and keeps kBT;
* total momentum is conserved; batch calls equal single-box calls bitwise;
* a cubic box under strong extension trips the CELL guard.
"""
import math

import numpy as np
import pytest

from paper_2512_13267_amd import inputs


def _box(orc, wl, k=0):
    b = wl.boxes[k]
    return orc.OracleBox(s=b.s, c=b.c, h=b.h, n_chains=b.n_chains, box_id=k)


def test_free_particles_move_straight_under_shear(orc):
    p = inputs.default_params(a=0.0, gamma=0.0, sigma=0.0)
    ell, rate = 5.0, 0.9
    rng = np.random.default_rng(8)
    N = 40
    h0 = np.diag([ell, ell, ell])
    s0 = rng.random((N, 3))
    c0 = rng.normal(size=(N, 3))
    c0 -= c0.mean(axis=0)  # every call starts from zero mean peculiar velocity
    L = inputs.shear_gradient(rate)
    r0 = s0 @ h0.T
    v0 = c0 + r0 @ L.T  # lab velocity = peculiar + streaming
    bx = orc.OracleBox(s=s0, c=c0, h=h0, n_chains=0)
    t = 0.0
    for chunk in range(8):
        orc.run_box(p, 1, 10, bx, L, 50)
        t += 50 * p["dt"]
        r = bx.s @ bx.h.T
        expect = r0 + t * v0
        # r and expect differ by a lattice vector of the current cell
        n = (expect - r) @ np.linalg.inv(bx.h).T
        assert np.allclose(n, np.round(n), atol=1e-9)
        # peculiar velocity: c(t) = (I - t L) c0 exactly
        assert np.allclose(bx.c, c0 - t * c0 @ L.T, atol=1e-12)
    assert bx.err == 0


def test_each_call_starts_from_zero_mean_peculiar_velocity(orc):
    """A call removes the box's mean peculiar velocity first: a state with a
    uniform offset continues exactly like the centred state (free particles
    under a compressing planar flow, where d<c>/dt = -L <c> would amplify
    the offset), and the mean stays zero."""
    p = inputs.default_params(a=0.0, gamma=0.0, sigma=0.0)
    rng = np.random.default_rng(9)
    N, ell = 30, 6.0
    h0 = np.diag([ell, ell, ell])
    s0 = rng.random((N, 3))
    c0 = rng.normal(size=(N, 3))
    c0 -= c0.mean(axis=0)
    L = inputs.planar_gradient(-0.3, 0.2, 0.0)
    a = orc.OracleBox(s=s0, c=c0, h=h0, n_chains=0)
    b = orc.OracleBox(s=s0, c=c0 + np.array([0.7, -0.4, 0.2]), h=h0, n_chains=0)
    for _ in range(3):
        orc.run_box(p, 1, 10, a, L, 40)
        orc.run_box(p, 1, 10, b, L, 40)
        assert np.abs(a.c - b.c).max() < 1e-12 and np.abs(a.s - b.s).max() < 1e-12
        assert np.abs(b.c.mean(axis=0)).max() < 1e-12


def test_energy_conserved_without_thermostat(orc):
    p = inputs.default_params(gamma=0.0, sigma=0.0, dt=0.005)
    wl = inputs.single_box(edge=5.0, polymer_fraction=0.2, shear_rate=0.0)
    bx = _box(orc, wl)

    def energy():
        ij, d = orc.pairs(bx.s, bx.h, 1.0, 0)
        r = np.linalg.norm(d, axis=1)
        U = np.sum(0.5 * p["a"] * (1 - r) ** 2)
        for ch in range(bx.n_chains):
            for k in range(9):
                i = ch * 10 + k
                ds = bx.s[i] - bx.s[i + 1]
                ds -= np.floor(ds + 0.5)
                x = bx.h @ ds
                U += -0.5 * p["H"] * p["R0"] ** 2 * np.log(1 - (x @ x) / p["R0"] ** 2)
        return U + 0.5 * p["mass"] * np.sum(bx.c ** 2)

    orc.run_box(p, 1, 10, bx, np.zeros((3, 3)), 100)  # leave the random start
    E0 = energy()
    Es = []
    for _ in range(10):
        orc.run_box(p, 1, 10, bx, np.zeros((3, 3)), 100)
        Es.append(energy())
    Es = np.array(Es)
    assert np.max(np.abs(Es - E0)) < 2e-4 * abs(E0)
    assert bx.err == 0


def test_equilibrium_temperature(orc):
    wl = inputs.single_box(edge=6.0, polymer_fraction=0.0, shear_rate=0.0)
    p = wl.params
    bx = _box(orc, wl)
    orc.run_box(p, p["seed"], 10, bx, np.zeros((3, 3)), 600)
    kts = []
    for _ in range(30):
        orc.run_box(p, p["seed"], 10, bx, np.zeros((3, 3)), 100)
        kts.append(np.sum(bx.c ** 2) / (3 * len(bx.c) - 3))
    kts = np.array(kts)
    se = kts.std(ddof=1) / math.sqrt(len(kts))
    assert abs(kts.mean() - 1.0) < max(3 * se, 0.02)
    assert se < 0.01


def test_dissipative_shear_viscosity_closed_form(orc):
    rate = 1.0
    wl = inputs.single_box(edge=6.0, polymer_fraction=0.0, shear_rate=rate, a=0.0)
    p = wl.params
    bx = _box(orc, wl)
    orc.run_box(p, p["seed"], 10, bx, wl.boxes[0].L, 400)
    vals = []
    for _ in range(30):
        _, parts, _ = orc.run_box(p, p["seed"], 10, bx, wl.boxes[0].L, 100)
        vals.append(parts[2, 3] / rate)  # dissipative part, xy
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    eta_d = 2 * math.pi * p["gamma"] * 3.0 ** 2 / 1575
    assert se < 0.05 * eta_d
    assert abs(vals.mean() - eta_d) < 3 * se + 0.01 * eta_d


def _solvent_shear(orc, rate, nsteps, n_rep=8, edge=6.0):
    """Block means (100 steps each, after 300 steps of start-up) of
    sigma_xy / rate, N1 = sigma_xx - sigma_yy and N2 = sigma_yy - sigma_zz,
    each averaged over n_rep independent solvent boxes of one batch call."""
    boxes, Ls = [], []
    for k in range(n_rep):
        wl = inputs.single_box(seed_k=40 + k, edge=edge, polymer_fraction=0.0, shear_rate=rate)
        boxes.append(_box(orc, wl))
        boxes[-1].box_id = k
        Ls.append(wl.boxes[0].L)
    p = wl.params
    orc.run_batch(p, p["seed"], p["chain_len"], boxes, Ls, 300)
    rows = []
    for _ in range(nsteps // 100):
        m, _ = orc.run_batch(p, p["seed"], p["chain_len"], boxes, Ls, 100)
        m = m.mean(axis=0)
        rows.append([m[3] / rate, m[0] - m[1], m[1] - m[2]])
    rows = np.array(rows)
    return rows.mean(axis=0), rows.std(axis=0, ddof=1) / math.sqrt(len(rows))


def test_newtonian_solvent_limit(orc):
    """Plain DPD solvent (a = 25, gamma = 4.5, density 3) in simple shear is
    a Newtonian fluid at these rates: its viscosity estimate does not depend
    on the rate and it has no normal-stress differences.  Longer runs at
    lower rates keep the standard error of sigma_xy / rate comparable
    (observed eta ~0.84 with SE 0.04-0.07)."""
    res = {rate: _solvent_shear(orc, rate, ns) for rate, ns in ((0.2, 2000), (0.1, 4000), (0.05, 8000))}
    rates = sorted(res)
    for r in rates:
        (eta, n1, n2), (se_eta, se1, se2) = res[r]
        print(f"rate {r}: eta {eta:.4f} +- {se_eta:.4f}, N1 {n1:.4f} +- {se1:.4f}, N2 {n2:.4f} +- {se2:.4f}")
        assert se_eta < 0.12 * eta
        assert abs(n1) < 2 * se1 and abs(n2) < 2 * se2
    for i in range(len(rates)):
        for j in range(i + 1, len(rates)):
            (ea, _, _), (sa, _, _) = res[rates[i]]
            (eb, _, _), (sb, _, _) = res[rates[j]]
            assert abs(ea - eb) < 2 * math.sqrt(sa * sa + sb * sb)
    # the conservative and kinetic parts raise the viscosity well above the
    # purely dissipative closed form of the a = 0 fluid (0.1616)
    assert all(res[r][0][0] > 2 * 0.1616 for r in rates)


def test_pure_rotation_no_deviatoric_stress(orc):
    om = 0.4
    wl = inputs.single_box(edge=6.0, polymer_fraction=0.1, shear_rate=0.0)
    L = inputs.planar_gradient(0.0, -om, om)
    p = wl.params
    bx = _box(orc, wl)
    orc.run_box(p, p["seed"], 10, bx, L, 400)
    dev, kts = [], []
    for _ in range(20):
        m, _, _ = orc.run_box(p, p["seed"], 10, bx, L, 100)
        tr = m[:3].mean()
        dev.append([m[0] - tr, m[1] - tr, m[3]])
        kts.append(np.sum(bx.c ** 2) / (3 * len(bx.c) - 3))
    dev = np.array(dev)
    se = dev.std(axis=0, ddof=1) / math.sqrt(len(dev))
    assert np.all(np.abs(dev.mean(axis=0)) < 4 * se + 0.05)
    assert abs(np.mean(kts) - 1.0) < 0.03
    assert bx.err == 0


def test_momentum_conserved_and_batch_equals_single(orc):
    wl = inputs.tiny_boxes(3)
    p = wl.params
    singles = [_box(orc, wl, k) for k in range(3)]
    batch = [_box(orc, wl, k) for k in range(3)]
    Ls = [b.L for b in wl.boxes]
    ms = [orc.run_box(p, p["seed"], 10, bx, L, 60)[0] for bx, L in zip(singles, Ls)]
    mb, _ = orc.run_batch(p, p["seed"], 10, batch, Ls, 60)
    for k in range(3):
        assert np.array_equal(singles[k].s, batch[k].s)
        assert np.array_equal(singles[k].c, batch[k].c)
        assert np.array_equal(ms[k], mb[k])
    # pair forces cancel, so the total peculiar momentum obeys dP/dt = -L P;
    # the call starts from P = 0 (mean removed), so it stays zero to rounding
    for k in range(3):
        assert abs(wl.boxes[k].c.sum(axis=0)).max() > 1e-8  # the generator's FP32 rounding left a residue
        P = singles[k].c.sum(axis=0)
        assert np.abs(P).max() < 1e-11 * len(singles[k].c)


def test_stretching_cube_trips_cell_guard(orc):
    wl = inputs.single_box(edge=4.2, polymer_fraction=0.0, shear_rate=0.0)
    p = wl.params
    bx = _box(orc, wl)
    L = inputs.planar_gradient(0.5, 0.0, 0.0)
    orc.run_box(p, p["seed"], 10, bx, L, 200)
    assert bx.err & orc.ERR_CELL


def test_bad_gradient_rejected(orc):
    wl = inputs.tiny_boxes(1)
    p = wl.params
    bx = _box(orc, wl)
    L = np.eye(3) * 0.1
    with pytest.raises(ValueError):
        orc.run_box(p, p["seed"], 10, bx, L, 5)
    assert bx.err & orc.ERR_ARG
