"""GPU checks of the LHMM step with the surrogate in the loop
(lhmm_hybrid_*), through the C ABI.

* all-DPD mode equals the coupled exchange interval (lhmm_couple_step, itself
  checked against the oracle) bit for bit;
* surrogate mode with a zero gate threshold sends every particle to DPD and
  equals all-DPD mode bit for bit (restore from the snapshot at the first
  step is the identity, subset steps of every box equal full steps);
* surrogate mode with the gate closed follows the oracle loop (SPH oracle,
  MLP oracle with the BF16 rounding points, feature and blend definitions)
  over several macro steps; the only differences are FP32 accumulation and
  BF16 rounding decisions in the ensemble (parity of the forward pass is
  ~1e-4 relative), which move the velocities by far less than 1e-6 of
  their scale over these steps.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as mo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(precision="fp32", n_particles=600, n_lattice=16, k_seed=11):
    from paper_2512_13267_amd import inputs, lhmm, micro

    mac = inputs.cylinder_array(n=n_lattice, force=2.0)
    q = mac.params
    nm = mac.r.shape[0] - q["n_fixed"]
    wl = inputs.lhmm_boxes(nm, n_particles=n_particles, polymer_fraction=0.2, seed_k=k_seed)
    m = micro.from_workload(wl, precision=precision)
    # the hybrid takes an equilibrated engine (forces of its current state
    # known): a few steps at rest
    import torch

    m.step(torch.zeros((m.n_boxes, 9), dtype=torch.float64, device="cuda"), 5)
    s = lhmm.Sph(q, mac.r, mac.v)
    return mac, q, wl, m, s


def test_dpd_mode_equals_coupled_interval_bitwise(torch_gpu):
    from paper_2512_13267_amd import lhmm

    mac, q, wl, m1, s1 = _setup()
    _, _, _, m2, s2 = _setup()
    cp = lhmm.Coupled(s1, m1)
    hy = lhmm.Hybrid(s2, m2, mode="dpd", k_micro=10)
    for _ in range(4):
        cp.step(10)
        st = hy.step()
        assert st["n_reset"] == 0
    sig1, _ = cp.coupling_state()
    sig2, _ = hy.state()
    r1, v1, _ = s1.get_state()
    r2, v2, _ = s2.get_state()
    assert np.array_equal(r1, r2) and np.array_equal(v1, v2)
    assert np.array_equal(sig1, sig2)
    hy.close()
    for e in (m1, s1, m2, s2):
        e.close()


def test_open_gate_sends_everything_to_dpd_bitwise(torch_gpu):
    from paper_2512_13267_amd import lhmm, surrogate

    outs = []
    for mode in ("dpd", "surrogate"):
        mac, q, wl, m, s = _setup()
        nm = m.n_boxes
        sur = None
        if mode == "surrogate":
            mem = surrogate.init_members(3, 129, 64, 3, seed=1)
            sur = surrogate.Surrogate(mem, 129, 64, 3, max_batch=nm)
        hy = lhmm.Hybrid(s, m, sur, phi=np.zeros(nm), mode=mode, k_micro=10, hold=1, replay=0,
                         threshold=0.0, floor=1e-6)
        for _ in range(3):
            st = hy.step()
        sig, on = hy.state()
        r, v, _ = s.get_state()
        assert on.all() and st["n_dpd"] == nm
        outs.append((sig, r, v))
        hy.close()
        m.close()
        s.close()
        if sur is not None:
            sur.close()
    (a, ra, va), (b, rb, vb) = outs
    assert np.array_equal(a, b) and np.array_equal(ra, rb) and np.array_equal(va, vb)


def test_closed_gate_follows_the_oracle_loop(torch_gpu, orc):
    from paper_2512_13267_amd import lhmm, surrogate

    mac, q, wl, m, s = _setup()
    n, nm = mac.r.shape[0], m.n_boxes
    E, nh = 3, 64
    members = surrogate.init_members(E, 129, nh, 3, seed=2)
    members = [{k: v.astype(np.float32).astype(np.float64) for k, v in mm.items()} for mm in members]
    sur = surrogate.Surrogate(members, 129, nh, 3, max_batch=nm)
    phi = np.full(nm, 0.5, dtype=np.float32)
    gscale, sscale = 8.0, 0.05
    hy = lhmm.Hybrid(s, m, sur, phi=phi, mode="surrogate", k_micro=10, hold=1, replay=0, threshold=1e30,
                     floor=1.0, grad_scale=gscale, stress_scale=sscale)
    r, v = mac.r.copy(), mac.v.copy()
    hist = np.zeros((nm, 32, 4))
    sigma = np.zeros((n, 6))
    for t in range(5):
        st = hy.step()
        assert st["n_dpd"] == 0 and st["micro_box_steps"] == 0
        pi = orc.sph_polymer_stress(q, sigma)
        L = orc.sph_step(q, r, v, pi)
        sample = np.stack([L[:nm, 0, 0], L[:nm, 0, 1], L[:nm, 1, 0], L[:nm, 1, 1]], axis=1) * gscale
        hist = np.concatenate([hist[:, 1:], sample.astype(np.float32).astype(np.float64)[:, None]], axis=1)
        X = mo.features(hist, phi.astype(np.float64))
        Ym = np.mean([mo.forward(mm, X)[0] for mm in members], axis=0)
        sigma = np.zeros((n, 6))
        sigma[:nm] = mo.blend(Ym, None, None, sscale)
    sig_d, on = hy.state()
    rg, vg, _ = s.get_state()
    assert not on.any()
    scale = np.abs(sigma).max()
    print("stress diff / scale", np.abs(sig_d - sigma).max() / scale, flush=True)
    assert np.abs(sig_d - sigma).max() < 2e-3 * scale
    assert not sig_d[nm:].any()
    dv = np.abs(vg - v).max() / np.abs(v).max()
    print("velocity diff / scale", dv, flush=True)
    assert dv < 1e-6
    hy.close()
    sur.close()
    m.close()
    s.close()
