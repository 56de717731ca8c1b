"""GPU parity of micro-domains with boundary regions (lhmm_micro_set_afbc;
Sec. "Macro-to-Micro Coupling", Eq. micro_bc, Tab. 2; core Irving-Kirkwood
stress) against the oracle (oracle_run_box_afbc), through the C ABI.

* FP64, the paper's planar melt (Tab. 1, N_d = 8) in a 28 x 28 cell with a
  core of half-width 4 and a ring out to 9, under simple shear and under
  planar extension: 200-step trajectories within 1e-4 and the core stress
  and its parts (kinetic, conservative, dissipative, random, FENE) to 1e-6
  of the stress scale;
* a batch mixing a boundary-region box with plain boxes: every box follows
  its own oracle (the variant kernel leaves plain boxes alone);
* the paper's micro-domain size, 76 x 76 (23,104 particles) with core 12
  and ring 25 (Tab. 2: 24 / 13 / 13), 40 FP64 steps against the oracle;
* bad regions are rejected.
"""
import numpy as np
import pytest

from paper_2512_13267_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _planar(edge, seed, chain_len=8):
    p = inputs.default_params(a=25.0, gamma=4.5, sigma=3.0, H=50.0, R0=1.5, dt=0.005, chain_len=chain_len,
                              seed=inputs.SEED_BASE + seed)
    rng = np.random.default_rng(inputs.SEED_BASE + seed)
    h = np.diag([edge, edge, inputs.PLANAR_THICKNESS])
    N = int(round(4.0 * edge * edge))
    nch = N // chain_len
    s, c = inputs.random_box(rng, h, N, nch, chain_len, planar=True)
    return p, h, s, c, nch


def _dr(s1, s2, h):
    ds = s1 - s2
    ds -= np.round(ds)
    return np.abs(ds @ np.asarray(h).T).max()


@pytest.mark.parametrize("flow", ["shear", "extension"])
def test_afbc_fp64_matches_oracle(torch_gpu, orc, flow):
    torch = torch_gpu
    from paper_2512_13267_amd import micro

    p, h, s, c, nch = _planar(28.0, 71)
    G = inputs.shear_gradient(0.2) if flow == "shear" else inputs.planar_gradient(0.05, 0.0, 0.0)
    print(f"case: AFBC 28 x 28 planar melt, {flow}, FP64, 200 steps", flush=True)
    m = micro.Micro(p, [(len(s), nch, h, 5)], precision="fp64", components=True)
    m.set_state(s, c, h, 0)
    m.set_afbc([[4.0, 9.0]], zeta=10.0)
    Gd = torch.tensor(G.reshape(1, 9), dtype=torch.float64, device="cuda")
    out = m.step(Gd, 200).cpu().numpy()[0]
    comps = m.components()[0]
    sd, cd, hd, st = m.get_state()
    box = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=5)
    mean, parts = orc.run_box_afbc(p, p["seed"], p["chain_len"], box, G, 4.0, 9.0, 200, zeta=10.0)
    assert st == box.step == 200
    assert np.allclose(hd[0], h, rtol=0, atol=0)  # the cell does not deform
    assert _dr(sd, box.s, h) <= 1e-4 and np.abs(cd - box.c).max() <= 1e-4
    scale = np.abs(mean).max()
    print("stress", out, "oracle", mean, flush=True)
    assert np.abs(out - mean).max() <= 1e-6 * scale
    assert np.abs(comps - parts).max() <= 1e-6 * scale
    m.close()


def test_afbc_box_beside_plain_boxes(torch_gpu, orc):
    torch = torch_gpu
    from paper_2512_13267_amd import micro

    p, h, s, c, nch = _planar(24.0, 72)
    wl = inputs.tiny_boxes(2, seed_k=73, **{k: p[k] for k in ("a", "gamma", "sigma", "H", "R0", "dt", "chain_len")})
    wl.params["seed"] = p["seed"]
    boxes = [(len(s), nch, h, 0)] + [(b.N, b.n_chains, b.h, k + 1) for k, b in enumerate(wl.boxes)]
    print("case: AFBC box + 2 plain boxes, FP64, 100 steps", flush=True)
    m = micro.Micro(p, boxes, precision="fp64")
    m.set_state(np.concatenate([s] + [b.s for b in wl.boxes]), np.concatenate([c] + [b.c for b in wl.boxes]),
                np.stack([h.reshape(9)] + [b.h.reshape(9) for b in wl.boxes]), 0)
    m.set_afbc([[3.0, 8.0], [0.0, 0.0], [0.0, 0.0]], zeta=10.0)
    Ls = [inputs.shear_gradient(0.1)] + [b.L for b in wl.boxes]
    out = m.step(torch.tensor(np.stack([L.reshape(9) for L in Ls]), dtype=torch.float64, device="cuda"), 100)
    out = out.cpu().numpy()
    sd, cd, hd, _ = m.get_state()
    off = np.concatenate([[0], np.cumsum([b[0] for b in boxes])])
    ob = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=0)
    mean0, _ = orc.run_box_afbc(p, p["seed"], p["chain_len"], ob, Ls[0], 3.0, 8.0, 100, zeta=10.0)
    assert np.abs(out[0] - mean0).max() <= 1e-6 * np.abs(mean0).max()
    assert _dr(sd[:off[1]], ob.s, h) <= 1e-4
    for k, b in enumerate(wl.boxes):
        o = orc.OracleBox(s=b.s, c=b.c, h=b.h, n_chains=b.n_chains, box_id=k + 1)
        mk, _, _ = orc.run_box(p, p["seed"], p["chain_len"], o, b.L, 100)
        assert np.abs(out[k + 1] - mk).max() <= 1e-6 * np.abs(mk).max(), k
        assert _dr(sd[off[k + 1]:off[k + 2]], o.s, o.h) <= 1e-4
        assert np.allclose(hd[k + 1], o.h, rtol=0, atol=1e-10)
    m.close()


def test_afbc_paper_domain_size(torch_gpu, orc):
    """76 x 76 at 4 particles per unit area (23,104, the paper's micro-domain
    of Tab. 2), core half-width 12, ring out to 25: 40 FP64 steps."""
    torch = torch_gpu
    from paper_2512_13267_amd import micro

    p, h, s, c, nch = _planar(76.0, 74)
    G = inputs.shear_gradient(0.05)
    print("case: AFBC 76 x 76 (23104 particles), FP64, 40 steps", flush=True)
    m = micro.Micro(p, [(len(s), nch, h, 9)], precision="fp64")
    m.set_state(s, c, h, 0)
    m.set_afbc([[12.0, 25.0]], zeta=10.0)
    out = m.step(torch.tensor(G.reshape(1, 9), dtype=torch.float64, device="cuda"), 40).cpu().numpy()[0]
    sd, cd, _, _ = m.get_state()
    box = orc.OracleBox(s=s, c=c, h=h, n_chains=nch, box_id=9)
    mean, _ = orc.run_box_afbc(p, p["seed"], p["chain_len"], box, G, 12.0, 25.0, 40, zeta=10.0)
    assert _dr(sd, box.s, h) <= 1e-4 and np.abs(cd - box.c).max() <= 1e-4
    assert np.abs(out - mean).max() <= 1e-6 * np.abs(mean).max()
    m.close()


def test_afbc_rejects_bad_regions(torch_gpu):
    from paper_2512_13267_amd import micro

    p, h, s, c, nch = _planar(20.0, 75)
    m = micro.Micro(p, [(len(s), nch, h, 0)], precision="fp32")
    m.set_state(s, c, h, 0)
    for bad in ([[5.0, 11.0]], [[6.0, 4.0]], [[-1.0, 3.0]], [[float("nan"), 3.0]]):
        with pytest.raises(Exception):
            m.set_afbc(bad, zeta=10.0)
    with pytest.raises(Exception):
        m.set_afbc([[3.0, 6.0]], zeta=-1.0)
    m.set_afbc([[3.0, 10.0]], zeta=0.0)
    m.close()
