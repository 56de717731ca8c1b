"""Virtual rheometer: the Carreau-Yasuda form and fit, the normal-stress
coefficient and relaxation time, pinned on closed forms (no GPU), and a
short shear sweep on the GPU."""
import math

import numpy as np
import pytest

from paper_2512_13267_amd import rheometer


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
