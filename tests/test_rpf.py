"""Reverse Poiseuille flow with the paper's macro set-up: the closed forms
and the set-up helpers pinned on the momentum balance (no GPU), the SPH
engine alone against the Newtonian steady parabola, and the coupled loop
against the exact steady shear stress (GPU)."""
import math

import numpy as np
import pytest

from paper_2512_13267_amd import inputs, rpf


@pytest.fixture(scope="module")
def torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_closed_forms_satisfy_the_momentum_balance():
    F, rho, eta, Ly = 0.01, 1.3, 0.05, 4.0
    y = np.linspace(0.0, Ly, 4001)
    tau = rpf.rpf_shear_stress(y, F, rho, Ly)
    v = rpf.rpf_velocity(y, F, rho, eta, Ly)
    f = np.where(y >= 0.5 * Ly, F, -F)
    dy = y[1] - y[0]
    inner = (np.abs(y - 0.5 * Ly) > 2 * dy) & (y > 2 * dy) & (y < Ly - 2 * dy)
    # steady balance d tau / dy = -rho f
    dtau = np.gradient(tau, dy)
    assert np.allclose(dtau[inner], -rho * f[inner], rtol=1e-9, atol=1e-12)
    # the Newtonian velocity carries that stress: eta dv/dy = tau, eta v'' = -rho f
    dv = np.gradient(v, dy)
    assert np.allclose(eta * dv[inner], tau[inner], rtol=0, atol=1e-6 * rho * F * Ly)
    d2v = np.gradient(dv, dy)
    assert np.allclose(eta * d2v[inner], -rho * f[inner], rtol=1e-6)
    # periodic, continuous, zero mean, peak rho F Ly / 4 at the switches
    assert tau[0] == pytest.approx(tau[-1]) and v[0] == pytest.approx(v[-1], abs=1e-15)
    assert rpf.rpf_shear_stress(0.5 * Ly - 1e-12, F, rho, Ly) == pytest.approx(
        rpf.rpf_shear_stress(0.5 * Ly, F, rho, Ly))
    assert abs(np.trapezoid(tau, y)) < 1e-9 and abs(np.trapezoid(v, y)) < 1e-9
    assert tau.max() == pytest.approx(rho * F * Ly / 4) and tau.min() == pytest.approx(-rho * F * Ly / 4)
    # peak speed F n Ly^2 / (32 eta) with n -> rho, upper stream along +x
    assert v.max() == pytest.approx(F * rho * Ly ** 2 / (32 * eta)) and v[np.argmax(v)] > 0
    assert y[np.argmax(v)] == pytest.approx(0.75 * Ly, abs=dy)


def test_startup_series_reaches_the_parabola_and_solves_the_diffusion_equation():
    F, rho, eta, Ly = 0.01, 1.0, 0.025, 4.0
    y = np.linspace(0.05, Ly - 0.05, 40)
    assert not rpf.rpf_startup_velocity(y, 0.0, F, rho, eta, Ly).any()
    late = rpf.rpf_startup_velocity(y, 1e5, F, rho, eta, Ly, n_modes=4000)
    assert np.abs(late - rpf.rpf_velocity(y, F, rho, eta, Ly)).max() < 1e-4 * F * rho * Ly ** 2 / (32 * eta)
    # v_t = nu v_yy + f away from the switches, by central differences
    yy = np.array([0.6, 1.0, 1.4, 2.6, 3.0, 3.4])
    t, dt, dy, nu = 7.0, 1e-3, 1e-3, eta / rho
    vt = (rpf.rpf_startup_velocity(yy, t + dt, F, rho, eta, Ly) - rpf.rpf_startup_velocity(yy, t - dt, F, rho, eta, Ly)) / (2 * dt)
    vyy = (rpf.rpf_startup_velocity(yy + dy, t, F, rho, eta, Ly) - 2 * rpf.rpf_startup_velocity(yy, t, F, rho, eta, Ly)
           + rpf.rpf_startup_velocity(yy - dy, t, F, rho, eta, Ly)) / dy ** 2
    f = np.where(yy >= 0.5 * Ly, F, -F)
    assert np.allclose(vt, nu * vyy + f, rtol=0, atol=2e-3 * F)


def test_sound_speed_and_cfl_limits():
    # each branch of Eq. (sound_speed) dominates in its own regime
    assert inputs.sound_speed(1.0, 1e-6, 1.0, 1e-6) == pytest.approx(10.0)
    assert inputs.sound_speed(1e-3, 1e3, 1.0, 1e-9) == pytest.approx(math.sqrt(1e3 * 1e-3 / 0.1))
    assert inputs.sound_speed(1e-6, 1e-6, 2.0, 5.0) == pytest.approx(math.sqrt(5.0 * 2.0 / 0.1))
    # each limit of Eq. (cfl_condition)
    assert inputs.cfl_dt(0.4, 0.1, 1.9, 0.0, 0.0) == pytest.approx(0.25 * 0.4 / 2.0)
    assert inputs.cfl_dt(0.4, 0.0, 1e-6, 100.0, 0.0) == pytest.approx(0.25 * math.sqrt(0.4 / 100.0))
    assert inputs.cfl_dt(0.4, 0.0, 1e-6, 0.0, 10.0) == pytest.approx(0.25 * 0.16 / 20.0)


def test_paper_set_up():
    m = inputs.reverse_poiseuille_paper()
    q = m.params
    assert m.n == 1600 and q["Lx"] == pytest.approx(4.0) and q["Ly"] == pytest.approx(4.0)
    assert q["kernel"] == inputs.KERNELS["lucy"] and q["h"] == pytest.approx(0.4)
    # delta_t = 0.32 = 8 x 0.04 = 64 x 0.005, within the CFL bound
    assert q["m_bar"] == 8 and q["k_micro"] == 64 and q["dt"] == pytest.approx(0.04) and q["dt"] <= q["dt_cfl"]
    assert q["theta"] > 0 and q["c"] > 0
    # the CFL step itself when none is given: M_bar rounds it down to a divisor of delta_t
    m2 = inputs.reverse_poiseuille_paper(force=1.0e-2, eta_p=0.0, dt_sph=None)
    q2 = m2.params
    assert q2["dt"] <= q2["dt_cfl"] and q2["m_bar"] * q2["dt"] == pytest.approx(0.32)
    assert (q2["m_bar"] - 1) * q2["dt_cfl"] < 0.32
    # Mach number near the delta = 0.1 of the sound-speed rule
    assert q["v_max"] / q["c"] <= 0.1 + 1e-12


@pytest.mark.gpu
def test_sph_alone_reaches_the_newtonian_parabola(torch_gpu):
    """SPH only (no polymer), the paper's macro set-up on a 10-column strip,
    time step from Eq. (cfl_condition): the start-up follows the Newtonian
    Fourier series, and after six start-up time constants the time-averaged
    velocity is the parabola of Appendix "Analytical velocity profile", both
    of the viscosity the SPH viscous term realises (5/4 eta_s); the velocity
    gradient carries the exact shear stress of Eq. RPF."""
    res = rpf.run(force=1.0e-2, alpha=0.0, eta_p_guess=0.0, nx=10, n_particles=0, startup=100.0, average=60.0,
                  log=None)
    print({k: res[k] for k in ("total_dev_rms", "total_dev_max", "vmax", "vmax_newtonian", "v_shape_rms",
                               "m_bar", "dt_sph", "seconds")})
    assert res["dt_sph"] <= res["dt_cfl"] and res["m_bar"] == 9
    assert res["vmax"] == pytest.approx(res["vmax_newtonian"], rel=0.03)
    # the start-up transient follows the Fourier series of the same viscosity
    mac = inputs.reverse_poiseuille_paper(force=1.0e-2, eta_p=0.0, alpha=0.0, nx=10)
    yrows = np.unique(mac.r[:, 1])
    for t, vmean in res["vmean_trace"][:12]:
        ref = np.abs(rpf.rpf_startup_velocity(yrows, t, 1.0e-2, 1.0, res["eta_sph"], 4.0)).mean()
        assert vmean == pytest.approx(ref, rel=0.03), (t, vmean, ref)
    assert res["v_shape_rms"] < 0.02
    assert res["total_dev_rms"] < 0.03 and res["total_dev_max"] < 0.05


@pytest.mark.gpu
def test_coupled_loop_reaches_the_exact_steady_stress(torch_gpu):
    """Coupled LHMM on a 20 x 40 strip of the paper's set-up, 800
    micro-boxes of 1000 particles: the time-averaged solvent plus polymer
    shear stress follows the exact triangle profile, the micro-domains carry
    a real share of it, and the velocity peak matches the Newtonian value
    of the total viscosity."""
    res = rpf.run(nx=20, n_particles=1000, startup=60.0, average=60.0, log=None)
    print({k: res[k] for k in ("total_dev_rms", "total_dev_max", "eta_p", "beta", "vmax", "vmax_newtonian",
                               "v_shape_rms", "seconds", "restored_boxes")})
    assert res["flagged_boxes"] == 0
    # measured: RMS 0.010, largest 0.020 of the peak stress; beta 0.43; peak
    # speed within 1.2 %, shape within 1.4 % (the micro stresses are noisy,
    # so the bounds leave about three times that)
    assert res["total_dev_rms"] < 0.03 and res["total_dev_max"] < 0.06
    assert 0.2 < res["beta"] < 0.8
    assert res["vmax"] == pytest.approx(res["vmax_newtonian"], rel=0.05)
    assert res["v_shape_rms"] < 0.04


@pytest.mark.gpu
def test_coupled_loop_with_the_papers_2d_melt(torch_gpu):
    """The paper's combination on a 20 x 40 strip: its macro set-up with
    planar micro-domains of its 2-D melt (Tab. 1, N_d = 8, 1024 particles
    each) and alpha = 2e-3 (its RPF case (c)); the total shear stress
    follows the exact profile and the melt carries a real share of it."""
    res = rpf.run(nx=20, n_particles=1024, micro_model="planar", chain_len=8, alpha=2.0e-3, eta_p_guess=0.026,
                  startup=60.0, average=60.0, lam=9.06, log=None)
    print({k: res[k] for k in ("total_dev_rms", "total_dev_max", "eta_p", "beta", "vmax", "vmax_newtonian",
                               "v_shape_rms", "seconds", "restored_boxes", "Re", "Wi")})
    assert res["flagged_boxes"] == 0
    assert res["total_dev_rms"] < 0.03 and res["total_dev_max"] < 0.06
    assert 0.2 < res["beta"] < 0.8
    assert res["vmax"] == pytest.approx(res["vmax_newtonian"], rel=0.05)
    assert res["v_shape_rms"] < 0.04


def test_run_rejects_an_unknown_micro_model():
    with pytest.raises(ValueError):
        rpf.run(micro_model="afbc", n_particles=10, log=None)


def test_planar_lhmm_boxes():
    wl = inputs.lhmm_boxes(2, n_particles=1024, density=4.0, polymer_fraction=1.0, seed_k=21, planar=True,
                           chain_len=8, dt=0.005)
    b = wl.boxes[0]
    assert b.N == 1024 and b.n_chains == 128 and np.allclose(np.diag(b.h), (16.0, 16.0, inputs.PLANAR_THICKNESS))
    assert not b.s[:, 2].any() and not b.c[:, 2].any()
    assert wl.params["H"] == 50.0 and wl.params["dt"] == 0.005 and wl.params["chain_len"] == 8
    # the 3-D recipe is unchanged
    w3 = inputs.lhmm_boxes(1, n_particles=300, polymer_fraction=0.2, seed_k=9)
    assert w3.params["H"] == 30.0 and w3.boxes[0].n_chains == 6 and w3.boxes[0].s[:, 2].any()


def test_report_lists_the_comparison():
    y = [0.1 + 0.2 * k for k in range(20)]
    n = len(y)
    res = {"workload": "w", "force": 0.01, "alpha": 0.002, "lambda_star": 1.0, "eta_s": 0.02, "eta_sph": 0.025,
           "c": 1.0, "theta": 0.5, "delta_t": 0.32, "m_bar": 8, "dt_sph": 0.04, "dt_cfl": 0.07, "k_micro": 64,
           "dt_micro": 0.005, "intervals": 376, "startup_intervals": 188, "samples": 47, "n_particles_total": 10,
           "seconds": 1.0, "replay": 10, "restored_boxes": 3, "flagged_boxes": 0, "total_dev_rms": 0.002,
           "total_dev_max": 0.004, "total_dev_rms_all": 0.003, "eta_p": 0.0155, "beta": 0.38, "U0": 0.084,
           "Re": 4.1, "Wi": 0.38, "lam": 9.06, "vmax": 0.1246, "vmax_newtonian": 0.1234, "v_shape_rms": 0.019,
           "y": y, "v": [0.0] * n, "v_ref": [0.0] * n, "solvent": [0.0] * n, "polymer": [0.0] * n,
           "total": [0.0] * n, "total_se": [0.0] * n, "tau_ref": [0.0] * n}
    text = rpf.report(res, "python -m paper_2512_13267_amd.rpf --micro planar")
    assert "Wi = 2 U0 lambda / L = 0.38" in text and "RMS deviation 0.002 tau_max" in text
    assert text.count("\n| ") == n + 1 and "(realised by the SPH viscous term as 0.025)" in text
    res["Wi"] = None
    assert "Wi =" not in rpf.report(res, "x")


@pytest.mark.parametrize("force,eta_p", [(1.8e-4, 0.0), (1.8e-4, 0.07), (1.0e-3, 0.02), (1.0e-2, 0.02),
                                         (1.0e-2, 0.07)])
def test_paper_forces_keep_the_papers_exchange_interval(force, eta_p):
    """The three body forces of the paper's reverse-Poiseuille table, with a
    polymer viscosity that keeps the flow within the CFL bound of the
    paper's step, give its interval 0.32 = 8 x 0.04 = 64 x 0.005; the sound
    speed keeps the Mach number at or below 0.1."""
    q = inputs.reverse_poiseuille_paper(force=force, eta_p=eta_p).params
    assert q["m_bar"] == 8 and q["dt"] == pytest.approx(0.04) and q["k_micro"] == 64
    assert q["dt"] <= q["dt_cfl"] and q["v_max"] / q["c"] <= 0.1 + 1e-12
