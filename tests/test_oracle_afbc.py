"""Pins of the oracle's micro-domain with boundary regions (Sec.
"Macro-to-Micro Coupling", Eq. micro_bc; Sec. "Micro-to-macro Coupling",
Eqs. IKtotal, kinetic_stress, potential_stress with a weight uniform over
the core; Tab. 2 regions).

* the bond function of a uniform core weight: the fraction of a segment
  inside the core square, against closed forms and against brute-force
  sampling of random segments;
* with the core covering the whole cell (and the ring empty), the domain
  is the plain periodic box: the same trajectory and the same stress
  times volume as the homogeneous-flow oracle at zero gradient;
* free particles (no forces, kBT = 0) on the boundary-condition ring relax
  toward the imposed field v' = G r' exactly as two half-step
  Ornstein-Uhlenbeck steps prescribe (and move with it when the rate is
  infinite), the others in straight lines; with kBT = 1 the ring's noise
  alone holds kBT;
* at zero imposed gradient the core's kinetic temperature is kBT per
  in-plane degree of freedom;
* under an imposed simple shear the core's mean velocity follows the
  imposed profile and the core's shear stress is positive.
"""
import math

import numpy as np
import pytest

from paper_2512_13267_amd import inputs


def test_core_fraction_closed_forms_and_sampling(orc):
    hc = 5.0
    assert orc.core_fraction([0, 0], [1, 2], hc) == 1.0
    assert orc.core_fraction([6, 0], [8, 3], hc) == 0.0
    assert orc.core_fraction([0, 0], [10, 0], hc) == pytest.approx(0.5, abs=1e-15)
    assert orc.core_fraction([-10, 1], [10, 1], hc) == pytest.approx(0.5, abs=1e-15)
    assert orc.core_fraction([4, 4], [6, 6], hc) == pytest.approx(0.5, abs=1e-15)  # through the corner
    assert orc.core_fraction([6, 4], [4, 6], hc) == pytest.approx(0.0, abs=1e-15)  # touches the corner only
    assert orc.core_fraction([5, -1], [5, 1], hc) == 1.0  # along the edge (closed square)
    rng = np.random.default_rng(3)
    t = (np.arange(200000) + 0.5) / 200000
    for _ in range(40):
        a, b = rng.uniform(-8, 8, size=2), rng.uniform(-8, 8, size=2)
        f = orc.core_fraction(a, b, hc)
        assert f == pytest.approx(orc.core_fraction(b, a, hc), abs=1e-14)
        p = a[None] + t[:, None] * (b - a)[None]
        inside = np.mean(np.all(np.abs(p) <= hc, axis=1))
        assert abs(f - inside) < 2e-5


def _planar(edge, n_chains_frac=1.0, seed=61, chain_len=8, **over):
    """A planar melt domain of the paper's Tab. 1 model (no solvent), square
    cell of side edge in the plane z = 0 of a cell of z edge 3.5."""
    p = inputs.default_params(a=25.0, gamma=4.5, sigma=3.0, H=50.0, R0=1.5, dt=0.005, chain_len=chain_len,
                              seed=inputs.SEED_BASE + seed)
    p.update(over)
    rng = np.random.default_rng(inputs.SEED_BASE + seed)
    h = np.diag([edge, edge, inputs.PLANAR_THICKNESS])
    N = int(round(4.0 * edge * edge))
    nch = int(n_chains_frac * N) // chain_len
    s, c = inputs.random_box(rng, h, N, nch, chain_len, planar=True)
    return p, h, s, c, nch


def test_whole_cell_core_is_the_periodic_box(orc):
    p, h, s, c, nch = _planar(12.0)
    a = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=3)
    b = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=3)
    hc = 6.0 + p["rc"]  # every pair's segment, images included, lies inside
    ma, pa = orc.run_box_afbc(p, p["seed"], p["chain_len"], a, np.zeros((3, 3)), hc, hc, 40)
    mb, pb, _ = orc.run_box(p, p["seed"], p["chain_len"], b, np.zeros((3, 3)), 40)
    assert np.array_equal(a.s, b.s) and np.array_equal(a.c, b.c) and a.step == b.step == 40
    Vc, V = 4 * hc * hc * h[2, 2], np.linalg.det(h)
    assert np.allclose(ma * Vc, mb * V, rtol=1e-12, atol=1e-12 * np.abs(mb * V).max())
    assert np.allclose(pa * Vc, pb * V, rtol=1e-12, atol=1e-12 * np.abs(pb * V).max())


def test_ring_relaxes_toward_the_imposed_field(orc):
    """No forces (a = gamma = sigma = 0, no bonds).  With kBT = 0 the ring's
    relaxation is deterministic: over one step a ring particle's in-plane
    velocity follows two half-step Ornstein-Uhlenbeck relaxations toward
    u = G r' (damping exp(-zeta dt / 2) each, u at the position of each half
    kick), its position the drift in between; a core or buffer particle keeps
    its velocity.  With zeta -> infinity the ring moves exactly with the
    imposed field."""
    hc, hb, rate = 3.0, 6.0, 0.4
    G = inputs.shear_gradient(rate)
    for zeta in (10.0, 1e9):
        p, h, s, c, _ = _planar(20.0, n_chains_frac=0.0, a=0.0, gamma=0.0, sigma=0.0, kBT=0.0)
        dt = p["dt"]
        box = orc.OracleBox(s=s, c=c, h=h, n_chains=0, box_id=0)
        c0 = box.c - box.c.mean(axis=0)
        r0 = (box.s[:, :2] - 0.5) * 20.0
        orc.run_box_afbc(p, p["seed"], p["chain_len"], box, G, hc, hb, 1, zeta=zeta)
        d = math.exp(-0.5 * zeta * dt)
        m0 = np.max(np.abs(r0), axis=1)
        ring = (m0 >= hc + 0.05) & (m0 < hb - 0.05)
        u0 = r0 @ G[:2, :2].T
        c1 = u0 + (c0[:, :2] - u0) * d
        r1 = r0 + dt * c1
        u1 = r1 @ G[:2, :2].T
        c2 = u1 + (c1 - u1) * d
        assert ring.sum() > 50
        assert np.allclose(box.c[ring, :2], c2[ring], rtol=0, atol=1e-12)
        free = m0 < hc - 0.05
        assert np.allclose(box.c[free], c0[free], rtol=0, atol=1e-14)
        if zeta > 1e6:
            assert np.allclose(box.c[ring, :2], u1[ring], rtol=0, atol=1e-12)
        assert not box.c[:, 2].any()  # planar: the ring acts in the plane only


def test_ring_noise_holds_kbt(orc):
    """No forces, no imposed gradient: the ring's Ornstein-Uhlenbeck steps
    alone bring its particles to kBT per in-plane degree of freedom; the
    noise pair of a half kick is a standard normal pair."""
    p, h, s, c, _ = _planar(20.0, n_chains_frac=0.0, a=0.0, gamma=0.0, sigma=0.0)
    box = orc.OracleBox(s=s * np.array([1.0, 1.0, 1.0]), c=np.zeros_like(c), h=h, n_chains=0, box_id=2)
    hc, hb = 2.0, 9.5  # nearly the whole cell is ring
    orc.run_box_afbc(p, p["seed"], p["chain_len"], box, np.zeros((3, 3)), hc, hb, 400, zeta=10.0)
    r = (box.s[:, :2] - 0.5) * 20.0
    ring = (np.max(np.abs(r), axis=1) >= hc) & (np.max(np.abs(r), axis=1) < hb)
    v2 = box.c[ring, :2] ** 2
    print("ring kBT", v2.mean(axis=0))
    assert np.allclose(v2.mean(axis=0), 1.0, atol=4 * math.sqrt(2.0 / ring.sum()))
    xi = np.array([orc.afbc_noise(p["seed"], i, 1, 17, 2) for i in range(4000)])
    assert np.abs(xi.mean(axis=0)).max() < 0.06 and np.abs(xi.var(axis=0) - 1).max() < 0.08
    assert abs(np.mean(xi[:, 0] * xi[:, 1])) < 0.06


def _core_stats(orc, rate, steps, blocks, edge=28.0, hc=4.0, hb=9.0):
    p, h, s, c, nch = _planar(edge, seed=62)
    G = inputs.shear_gradient(rate)
    box = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=1)
    orc.run_box_afbc(p, p["seed"], p["chain_len"], box, G, hc, hb, 1600)  # past the start-up heating
    kts, sxy, prof = [], [], []
    for _ in range(blocks):
        m, parts = orc.run_box_afbc(p, p["seed"], p["chain_len"], box, G, hc, hb, steps)
        r = (box.s[:, :2] - 0.5) * edge
        core = np.max(np.abs(r), axis=1) < hc
        dv = box.c[core, :2] - r[core] @ G[:2, :2].T
        kts.append(np.mean(dv ** 2))
        sxy.append(m[3] * h[2, 2])  # 2-D stress
        prof.append(np.polyfit(r[core, 1], box.c[core, 0], 1)[0])
    return np.array(kts), np.array(sxy), np.array(prof)


def test_core_temperature_at_rest(orc):
    kts, sxy, _ = _core_stats(orc, 0.0, 100, 12)
    se = kts.std(ddof=1) / math.sqrt(len(kts))
    print("core kBT", kts.mean(), "+-", se)
    assert abs(kts.mean() - 1.0) < max(3 * se, 0.03)


def test_core_follows_imposed_shear(orc):
    rate = 0.2
    kts, sxy, slope = _core_stats(orc, rate, 100, 12)
    print("core velocity slope", slope.mean(), "+-", slope.std(ddof=1) / math.sqrt(len(slope)), "rate", rate,
          "core sigma_xy", sxy.mean())
    assert abs(slope.mean() - rate) < 0.15 * rate
    assert sxy.mean() > 0
    assert abs(kts.mean() - 1.0) < 0.1
