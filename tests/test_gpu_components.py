"""Stress by force type (Eqs. IKtotal, kinetic_stress, potential_stress with
the conservative, dissipative and random forces of Eqs. conservative,
dissipative, random kept apart, and the FENE bonds of Eq. fene_force), the
cumulative pair counter and graph preparation, through the C ABI.

* FP64 components of ragged boxes equal the oracle's parts to 1e-6 of the
  stress scale (rounding order only), and sum to the returned stress;
* the components variant gives the same trajectory, bit for bit, and the
  same stress as the default kernel (its pair sum is accumulated the same
  way);
* the device's dissipative part of a purely dissipative fluid (a = 0) under
  shear equals the closed form eta_D = 2 pi gamma rho^2 rc^5 / 1575 within
  three standard errors (FP32, the benchmark's precision);
* the cumulative pair counter adds up the per-call counts;
* preparing the graphs of a call changes nothing in its results.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _grads(torch, wl):
    return torch.tensor(np.stack([b.L for b in wl.boxes]), dtype=torch.float64, device="cuda").contiguous()


def test_components_match_oracle_fp64(torch_gpu, orc):
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    wl = inputs.tiny_boxes(5)
    p = wl.params
    print("case: 5 ragged boxes, FP64, 60 steps, components", flush=True)
    m = micro.from_workload(wl, precision="fp64", components=True)
    G = _grads(torch, wl)
    out = m.step(G, 60).cpu().numpy()
    comps = m.components()
    obs = [orc.OracleBox(s=b.s, c=b.c, h=b.h, n_chains=b.n_chains, box_id=k) for k, b in enumerate(wl.boxes)]
    means, parts = orc.run_batch(p, p["seed"], p["chain_len"], obs, [b.L for b in wl.boxes], 60)
    for k in range(len(wl.boxes)):
        scale = np.abs(means[k]).max()
        assert np.abs(comps[k] - parts[k]).max() <= 1e-6 * scale, k
        assert np.abs(comps[k].sum(axis=0) - out[k]).max() <= 1e-12 * scale
        # the random and dissipative parts are not negligible here
        assert np.abs(parts[k][2]).max() > 1e-3 * scale and np.abs(parts[k][3]).max() > 1e-3 * scale
    # without the option the engine refuses the call
    m0 = micro.from_workload(wl, precision="fp64")
    with pytest.raises(Exception):
        m0.components()
    out0 = m0.step(G, 60).cpu().numpy()
    s1, c1, h1, st1 = m.get_state()
    s0, c0, h0, st0 = m0.get_state()
    assert np.array_equal(s1, s0) and np.array_equal(c1, c0) and st1 == st0
    assert np.abs(out0 - out).max() <= 1e-13 * np.abs(out0).max()
    m.close()
    m0.close()


def test_components_fp32_trajectory_equals_default_kernel(torch_gpu):
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    wl = inputs.tiny_boxes(4, seed_k=9)
    print("case: 4 ragged boxes, FP32, 40 steps, components vs default", flush=True)
    G = _grads(torch, wl)
    m = micro.from_workload(wl, precision="fp32", components=True)
    m0 = micro.from_workload(wl, precision="fp32")
    out = m.step(G, 40).cpu().numpy()
    out0 = m0.step(G, 40).cpu().numpy()
    s1, c1, _, _ = m.get_state()
    s0, c0, _, _ = m0.get_state()
    assert np.array_equal(s1, s0) and np.array_equal(c1, c0)
    assert np.abs(out0 - out).max() <= 1e-12 * np.abs(out0).max()
    comps = m.components()
    # each part is summed in single precision per lane on its own
    assert np.abs(comps.sum(axis=1) - out).max() <= 1e-6 * np.abs(out).max()
    m.close()
    m0.close()


def test_dissipative_part_closed_form_on_device(torch_gpu):
    """a = 0, no chains, simple shear at rate 1: with g(r) = 1 the
    dissipative shear stress is eta_D * rate, eta_D = 2 pi gamma rho^2 rc^5 /
    1575 = 0.1616 at rho = 3, gamma = 4.5 (pair density rho^2/2, angular
    mean of e_x^2 e_y^2 = 1/15, int r^4 (1 - r)^2 dr = 1/105)."""
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    rate = 1.0
    wl = inputs.single_box(edge=8.0, polymer_fraction=0.0, shear_rate=rate, a=0.0)
    print("case: a = 0 solvent, 1536 particles, shear 1.0, FP32, components", flush=True)
    m = micro.from_workload(wl, precision="fp32", components=True)
    G = _grads(torch, wl)
    m.step(G, 400)
    vals = []
    for _ in range(40):
        m.step(G, 100)
        vals.append(m.components()[0, 2, 3] / rate)
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    eta_d = 2 * math.pi * wl.params["gamma"] * 3.0 ** 2 / 1575
    print("eta_D device", vals.mean(), "+-", se, "closed form", eta_d)
    assert se < 0.05 * eta_d
    assert abs(vals.mean() - eta_d) < 3 * se + 0.01 * eta_d
    m.close()


def test_pair_total_adds_up_the_calls(torch_gpu):
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    wl = inputs.tiny_boxes(3, seed_k=11)
    m = micro.from_workload(wl, precision="fp32")
    G = _grads(torch, wl)
    assert not m.pair_total().any()
    m.step(G, 10)
    c1 = m.pair_counts().copy()
    m.step(G, 7)
    c2 = m.pair_counts().copy()
    m.step_subset(G, 5, [1])
    c3 = m.pair_counts().copy()
    assert c1.min() > 0 and c2.min() > 0 and c3[1] > 0 and c3[0] == 0 and c3[2] == 0
    assert np.array_equal(m.pair_total(), c1 + c2 + c3)
    m.close()


def test_prepare_changes_no_result(torch_gpu):
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    wl = inputs.tiny_boxes(3, seed_k=12)
    G = _grads(torch, wl)
    a = micro.from_workload(wl, precision="fp32")
    b = micro.from_workload(wl, precision="fp32")
    a.prepare(73)  # a 50-step graph and a 23-step graph
    oa = a.step(G, 73).cpu().numpy()
    ob = b.step(G, 73).cpu().numpy()
    assert np.array_equal(oa, ob)
    sa, ca, _, _ = a.get_state()
    sb, cb, _, _ = b.get_state()
    assert np.array_equal(sa, sb) and np.array_equal(ca, cb)
    with pytest.raises(Exception):
        a.prepare(0)
    a.close()
    b.close()
