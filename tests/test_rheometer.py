"""Virtual rheometer: the Carreau-Yasuda form and fit, the normal-stress
coefficient and relaxation time, pinned on closed forms (no GPU), and a
short shear sweep on the GPU."""
import math

import numpy as np
import pytest

from paper_2512_13267_amd import inputs, rheometer


@pytest.fixture(scope="module")
def torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_carreau_yasuda_limits_and_special_cases():
    g = np.logspace(-4, 4, 41)
    # n = 1: Newtonian at eta0 for every rate
    assert np.allclose(rheometer.carreau_yasuda(g, 7.0, 1.0, 3.0, 0.8, 1.0), 7.0, rtol=0, atol=1e-12)
    # rate -> 0: eta0; rate -> infinity with n < 1: eta_inf
    assert rheometer.carreau_yasuda(1e-12, 34.29, 3.15, 89.75, 0.95, 0.37) == pytest.approx(34.29, rel=1e-9)
    assert rheometer.carreau_yasuda(1e12, 34.29, 3.15, 89.75, 0.95, 0.37) == pytest.approx(3.15, rel=1e-6)
    # a = 2, eta_inf = 0: the Carreau model eta0 (1 + (lam g)^2)^((n - 1) / 2)
    ref = 5.0 * (1.0 + (0.7 * g) ** 2) ** ((0.4 - 1.0) / 2.0)
    assert np.allclose(rheometer.carreau_yasuda(g, 5.0, 0.0, 0.7, 2.0, 0.4), ref, rtol=1e-12)
    # power-law regime: slope n - 1 in log-log well above 1 / lam, eta_inf = 0
    e = rheometer.carreau_yasuda(np.array([1e3, 1e4]), 10.0, 0.0, 1.0, 1.5, 0.3)
    assert math.log10(e[1] / e[0]) == pytest.approx(0.3 - 1.0, abs=1e-3)


def test_fit_recovers_known_parameters():
    g = np.logspace(-3, 1, 12)
    for truth in ((34.29, 3.15, 89.75, 0.95, 0.37), (13.2, 0.5, 23.5, 0.71, 0.6), (5.0, 0.8, 2.0, 2.0, 0.2)):
        eta = rheometer.carreau_yasuda(g, *truth)
        fit = rheometer.fit_carreau_yasuda(g, eta)
        assert fit["rms_rel_residual"] < 1e-6, (truth, fit)
        # the viscosity curve is recovered; eta0 and lam are well determined
        assert fit["eta0"] == pytest.approx(truth[0], rel=1e-3)
        assert fit["lam"] == pytest.approx(truth[2], rel=2e-2)
        assert fit["at_bounds"] == []
    # noisy data: parameters within a few per cent
    rng = np.random.default_rng(5)
    truth = (20.0, 2.0, 10.0, 1.0, 0.4)
    g = np.logspace(-3, 1, 16)
    eta = rheometer.carreau_yasuda(g, *truth) * (1.0 + 0.01 * rng.standard_normal(g.size))
    fit = rheometer.fit_carreau_yasuda(g, eta)
    assert fit["eta0"] == pytest.approx(20.0, rel=0.03)
    assert fit["rms_rel_residual"] < 0.02
    with pytest.raises(ValueError):
        rheometer.fit_carreau_yasuda(g[:4], eta[:4])
    # a curve that keeps thinning as 1 / rate (n = 0 exactly) puts n on its bound
    g = np.logspace(-2, 2, 12)
    fit = rheometer.fit_carreau_yasuda(g, rheometer.carreau_yasuda(g, 10.0, 0.5, 3.0, 2.0, 0.0))
    assert "n" in fit["at_bounds"] and fit["n"] == pytest.approx(0.0, abs=1e-4)


def test_normal_stress_and_relaxation_of_a_maxwell_fluid():
    # upper-convected Maxwell fluid (modulus G, relaxation time lam) in steady
    # simple shear: sigma_xy = G lam g, N1 = 2 G lam^2 g^2, so psi1 = 2 G lam^2
    # and 0.5 psi1 / eta = lam at every rate
    G, lam = 3.0, 7.5
    g = np.array([0.01, 0.1, 1.0])
    sigma = np.zeros((3, 6))
    sigma[:, 3] = G * lam * g
    sigma[:, 0] = 2.0 * G * lam ** 2 * g ** 2
    eta, n1, psi1, lam_g = rheometer.normal_stress_and_relaxation(g, sigma)
    assert np.allclose(eta, G * lam) and np.allclose(psi1, 2.0 * G * lam ** 2)
    assert np.allclose(lam_g, lam) and np.allclose(n1, sigma[:, 0])


def test_chain_scaling_and_report():
    n = np.array([5, 10, 20, 40])
    sc = rheometer.chain_scaling(n, 0.3 * n ** 1.9)
    assert sc["b"] == pytest.approx(1.9, abs=1e-12) and sc["prefactor"] == pytest.approx(0.3, rel=1e-12)
    rates = [0.01, 0.03, 0.1, 0.3, 1.0]
    fake = []
    for nd, lam in ((10, 5.0), (20, 20.0)):
        eta = rheometer.carreau_yasuda(np.array(rates), 5.0, 1.0, lam, 1.5, 0.4)
        fake.append({"rates": rates, "eta": eta.tolist(), "eta_se": (0.01 * eta).tolist(), "N1": [0.1] * 5,
                     "N1_se": [0.01] * 5, "psi1": [1.0] * 5, "lambda": [1.0] * 5, "chain_len": nd, "edge": 10.0,
                     "replicas": 16, "equil_steps": 10, "avg_steps": 10, "n_particles": 1, "seconds": 0.0,
                     "flagged_boxes": 0, "carreau_yasuda": rheometer.fit_carreau_yasuda(rates, eta)})
    text = rheometer.report(fake, "python -m paper_2512_13267_amd.rheometer")
    assert "b = 2.000" in text and "N_d = 20" in text


def test_sweep_workload_layout():
    wl = rheometer.sweep_workload([0.1, 1.0], replicas=3, chain_len=8, edge=5.0)
    assert len(wl.boxes) == 6 and wl.params["chain_len"] == 8
    assert all(b.n_chains * 8 <= b.N for b in wl.boxes)
    assert [b.L[0, 1] for b in wl.boxes] == [0.1] * 3 + [1.0] * 3
    # replicas start from different states
    assert not np.array_equal(wl.boxes[0].s, wl.boxes[1].s)


def test_planar_melt_stays_in_its_plane_at_kBT(orc):
    """The paper's 2-D melt (Tab. 1, n = 4, N_d = 8) held in the plane z = 0
    of a periodic cell: every z separation is zero, so positions and
    velocities never leave the plane (exactly), and the fluctuation-
    dissipation balance gives kBT per in-plane degree of freedom (time
    average of the kinetic stress, 2 %)."""
    wl = rheometer.sweep_workload([0.0, 0.05], replicas=1, chain_len=8, edge=6.0, density=4.0, planar=True)
    p = wl.params
    assert p["H"] == 50.0 and p["dt"] == 0.005 and wl.boxes[0].N == 144 and wl.boxes[0].n_chains == 18
    for k, b in enumerate(wl.boxes):
        assert not b.s[:, 2].any() and not b.c[:, 2].any()
        ob = orc.OracleBox(s=b.s, c=b.c, h=b.h, n_chains=b.n_chains, box_id=k)
        orc.run_box(p, p["seed"], 8, ob, b.L, 400)
        mean, parts, _ = orc.run_box(p, p["seed"], 8, ob, b.L, 3000)
        assert not ob.s[:, 2].any() and not ob.c[:, 2].any() and ob.err == 0
        V = float(np.linalg.det(ob.h))
        Tx, Ty, Tz = (-parts[0][:3] * V / b.N).tolist()
        assert Tz == 0.0 and mean[4] == 0.0 and mean[5] == 0.0
        if k == 0:
            assert Tx == pytest.approx(1.0, abs=0.02) and Ty == pytest.approx(1.0, abs=0.02)
    with pytest.raises(ValueError):
        inputs.random_box(np.random.default_rng(0), np.array([[5.0, 0, 1.0], [0, 5.0, 0], [0, 0, 3.5]]), 10, 0, 8,
                          planar=True)


@pytest.mark.gpu
def test_planar_melt_matches_oracle_and_sweeps(torch_gpu, orc):
    """FP64 planar boxes on the device against the oracle (200 steps, the
    tolerances of the 3-D trajectory tests), then a short FP32 planar sweep
    at the paper's parameters: positive viscosity, in-plane stress only."""
    from paper_2512_13267_amd import micro

    torch = torch_gpu
    wl = rheometer.sweep_workload([0.05, 0.5], replicas=1, chain_len=8, edge=8.0, density=4.0, planar=True)
    p = wl.params
    m = micro.from_workload(wl, precision="fp64", graphs=False)
    G = torch.tensor(np.stack([b.L for b in wl.boxes]), dtype=torch.float64, device="cuda").contiguous()
    out = m.step(G, 200).cpu().numpy()
    s, c, h, _ = m.get_state()
    obs = [orc.OracleBox(s=b.s, c=b.c, h=b.h, n_chains=b.n_chains, box_id=k) for k, b in enumerate(wl.boxes)]
    means, _ = orc.run_batch(p, p["seed"], 8, obs, [b.L for b in wl.boxes], 200)
    n = wl.boxes[0].N
    for k, ob in enumerate(obs):
        sk = s[k * n:(k + 1) * n]
        d = sk - ob.s
        d -= np.round(d)
        assert np.abs(d @ ob.h.T).max() <= 1e-4, k
        assert np.abs(c[k * n:(k + 1) * n] - ob.c).max() <= 1e-4, k
        assert np.abs(out[k] - means[k]).max() <= 1e-6 * np.abs(means[k]).max(), k
        assert not sk[:, 2].any() and not c[k * n:(k + 1) * n, 2].any()
    assert not m.flags().any()
    m.close()
    res = rheometer.run_sweep([0.05, 0.5], replicas=4, chain_len=8, equil=400, steps=800, edge=16.0, planar=True,
                              log=lambda *a, **k: None)
    assert res["dims"] == 2 and res["flagged_boxes"] == 0
    assert all(e > 0 for e in res["eta"]), res["eta"]
    sig = np.asarray(res["sigma_mean"])
    assert np.abs(sig[:, 4:]).max() == 0.0


@pytest.mark.gpu
def test_short_shear_sweep_on_gpu(torch_gpu):
    res = rheometer.run_sweep([0.5, 1.0, 2.0], replicas=4, chain_len=10, equil=300, steps=600, edge=6.0,
                              log=lambda *a, **k: None)
    eta = np.asarray(res["eta"])
    assert np.all(np.isfinite(eta)) and np.all(eta > 0), res
    # at these rates the signal is many standard errors above the noise
    assert np.all(eta > 3.0 * np.asarray(res["eta_se"])), res
    # a sheared polymer melt has a positive first normal stress difference
    assert res["N1"][-1] > 0.0, res
    assert res["flagged_boxes"] >= 0


def test_planar_report_compares_with_the_papers_table():
    rates = [0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0]
    eta = rheometer.carreau_yasuda(np.array(rates), 12.9, 3.2, 9.0, 1.5, 0.2)
    r = {"rates": rates, "eta": eta.tolist(), "eta_se": (0.01 * eta).tolist(), "N1": [0.1] * 8, "N1_se": [0.01] * 8,
         "psi1": [1.0] * 8, "lambda": [1.0] * 8, "chain_len": 8, "edge": 32.0, "dims": 2, "density": 4.0,
         "replicas": 16, "equil_steps": 10, "avg_steps": 10, "n_particles": 1, "seconds": 0.0, "flagged_boxes": 0,
         "carreau_yasuda": rheometer.fit_carreau_yasuda(rates, eta)}
    text = rheometer.report([r], "python -m paper_2512_13267_amd.rheometer --planar")
    assert "2-D melt" in text and "Tab. yasuda_params" in text and "34.29" in text
    assert "| 8 | 12.9" in text
    assert rheometer.PAPER_CY[8] == (34.29, 3.15, 89.75, 0.95, 0.37)
