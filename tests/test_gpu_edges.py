"""Edge cases and error paths of every engine through the C ABI (GPU):
degenerate boxes, extreme sizes and rejected arguments.  Every rejected
call must return an error code and leave the engine usable."""
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


def test_solvent_only_chain_only_and_single_particle_boxes(torch_gpu, orc):
    """Boxes with no chains, with every particle in chains, and a box whose
    two particles are farther apart than the cutoff: forces against the
    oracle.  A box of one particle is refused."""
    torch = torch_gpu
    from paper_2512_13267_amd import inputs, micro

    p = inputs.default_params(seed=inputs.SEED_BASE + 61)
    rng = np.random.default_rng(61)
    boxes = []
    for edge, N, nch in ((5.0, 375, 0), (5.0, 370, 37), (4.0, 2, 0), (4.5, 40, 0)):
        h = inputs.cubic_cell(edge)
        s, c = inputs.random_box(rng, h, N, nch, p["chain_len"], p["kBT"], p["mass"])
        if N == 2:
            s = np.array([[0.125, 0.125, 0.125], [0.625, 0.625, 0.625]])
        boxes.append(inputs.BoxInit(s=s, c=c, h=h, n_chains=nch, L=inputs.planar_gradient(0.1, 0.2, -0.1), edge=edge))
    from paper_2512_13267_amd import _lib

    with pytest.raises(_lib.LhmmError):
        micro.Micro(p, [(1, 0, inputs.cubic_cell(4.0))])
    wl = inputs.Workload("edges", p, boxes, 0)
    m = micro.from_workload(wl, precision="fp64")
    Ls = np.stack([b.L for b in boxes])
    f, vir = m.forces(Ls)
    off = np.concatenate([[0], np.cumsum([b.N for b in boxes])])
    for k, b in enumerate(boxes):
        Fr, Wr, err = orc.forces(p, p["seed"], p["chain_len"], k, b.n_chains, b.s, b.c, b.h, b.L, 0)
        Fg = f[off[k]:off[k + 1]]
        assert np.abs(Fg - Fr).max() <= 1e-10 * max(1.0, np.abs(Fr).max()), k
    out = m.step(_grads(torch, wl), 10).cpu().numpy()
    assert np.all(np.isfinite(out))
    assert m.pair_counts()[2] == 0
    m.close()


def test_micro_rejects_bad_arguments_and_stays_usable(torch_gpu):
    torch = torch_gpu
    from paper_2512_13267_amd import _lib, inputs, micro

    wl = inputs.tiny_boxes(2, seed_k=63)
    G = _grads(torch, wl)
    m = micro.from_workload(wl, precision="fp32")
    for bad in ([], [1, 0], [0, 0], [2], [-1]):
        with pytest.raises(_lib.LhmmError) as ei:
            m.step_subset(G, 5, bad)
        assert ei.value.code == _lib.LHMM_ERR_ARG
    with pytest.raises(_lib.LhmmError):
        m.restore([0])  # no snapshot yet
    for kw in ({"bin_threads": 128}, {"graph_chunk": 0}, {"queue_depth": 8, "drain": 7}, {"queue_depth": 12},
               {"prune": 2}, {"busy_lanes": 0}):
        with pytest.raises(_lib.LhmmError):
            m.set_config(**kw)
    out = m.step(G, 5).cpu().numpy()
    assert np.all(np.isfinite(out))
    m.close()
    # a box whose grid would exceed the per-box cell capacity is refused at create
    p = inputs.default_params()
    with pytest.raises(_lib.LhmmError):
        micro.Micro(p, [(10, 0, inputs.cubic_cell(40.0))])


def test_sph_surrogate_and_hybrid_reject_bad_arguments(torch_gpu):
    torch = torch_gpu
    from paper_2512_13267_amd import _lib, inputs, lhmm, micro, surrogate

    mac = inputs.cylinder_array(n=16)
    q = dict(mac.params)
    with pytest.raises(_lib.LhmmError):
        lhmm.Sph(dict(q, n_fixed=mac.r.shape[0]), mac.r, mac.v)  # no mobile particle
    with pytest.raises(_lib.LhmmError):
        lhmm.Sph(dict(q, force_mode=7), mac.r, mac.v)
    with pytest.raises(_lib.LhmmError, match="kernel"):
        lhmm.Sph(dict(q, kernel=2), mac.r, mac.v)
    r_out = mac.r.copy()
    r_out[0, 0] = 1.5
    with pytest.raises(_lib.LhmmError):
        lhmm.Sph(q, r_out, mac.v)
    members = surrogate.init_members(2, 129, 64, 3, seed=1)
    for E_nh in ((0, 64), (2, 48)):
        with pytest.raises((_lib.LhmmError, ValueError)):
            surrogate.Surrogate(members[:E_nh[0]] if E_nh[0] else [], 129, E_nh[1], 3, max_batch=8)
    s = surrogate.Surrogate(members, 129, 64, 3, max_batch=8)
    X = torch.zeros((33, 129), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.LhmmError):
        s.forward(X)  # batch above max_batch (8, rounded up to 32 rows)
    bad = [dict(m) for m in members]
    bad[0]["W2"] = bad[0]["W2"].copy()
    bad[0]["W2"][0, 0] = np.nan
    with pytest.raises(_lib.LhmmError):
        s.set_weights(bad)
    Y = s.forward(X[:8].contiguous())
    assert torch.isfinite(Y).all()
    nm = mac.r.shape[0] - q["n_fixed"]
    wl = inputs.lhmm_boxes(nm - 1, n_particles=300, seed_k=3)
    m = micro.from_workload(wl, precision="fp32")
    sph = lhmm.Sph(q, mac.r, mac.v)
    with pytest.raises(_lib.LhmmError):
        lhmm.Hybrid(sph, m, s, mode="dpd")  # one box short
    m.close()
    wl = inputs.lhmm_boxes(nm, n_particles=300, seed_k=3)
    m = micro.from_workload(wl, precision="fp32")
    with pytest.raises(_lib.LhmmError):
        lhmm.Hybrid(sph, m, s, mode="surrogate")  # surrogate batch too small
    with pytest.raises(_lib.LhmmError):
        lhmm.Hybrid(sph, m, None, mode="surrogate")
    with pytest.raises(_lib.LhmmError):
        lhmm.Hybrid(sph, m, None, mode="dpd", replay=32)
    hy = lhmm.Hybrid(sph, m, None, mode="dpd", k_micro=2)
    st = hy.step()
    assert st["n_dpd"] == nm and st["macro_step"] == 1
    hy.close()
    for e in (m, sph, s):
        e.close()
