"""GPU parity of the stress surrogate (lhmm_sur_*) against the float64 MLP
oracle, through the C ABI.

Tolerances.  Both sides round the same operands to BF16 and the oracle
computes everything else in float64; the device accumulates in FP32 and
evaluates GELU in FP32.  An FP32 pre-activation that lies within an FP32
rounding of a BF16 rounding boundary can round to the neighbouring BF16
value (one BF16 ulp, 2^-8 relative) on one side only, which moves the
product that consumes it by about 2^-8 |x w|.  The checks therefore bound
(a) the relative Frobenius error of each output or gradient block at 1e-3,
far above FP32 accumulation error (~1e-6) and far below a wrong term (O(1)),
and (b) the largest single error at 2^-6 of the block's scale.
"""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as mo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2512_13267_amd import surrogate as sur
    return sur


def _members(E, nin, nh, nout, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(E):
        out.append({"W1": rng.normal(scale=np.sqrt(2 / nin), size=(nin, nh)), "b1": rng.normal(scale=0.1, size=nh),
                    "W2": rng.normal(scale=np.sqrt(2 / nh), size=(nh, nh)), "b2": rng.normal(scale=0.1, size=nh),
                    "W3": rng.normal(scale=np.sqrt(1 / nh), size=(nh, nout)), "b3": rng.normal(scale=0.1, size=nout)})
    # the device holds FP32 masters: give the oracle the same FP32 values
    return [{k: v.astype(np.float32).astype(np.float64) for k, v in m.items()} for m in out]


def _data(B, nin, nout, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, nin)).astype(np.float32)
    T = (np.tanh(X[:, :nout] * 0.7) + 0.1 * rng.normal(size=(B, nout))).astype(np.float32)
    return X, T


def _close(dev, ref, what):
    dev = np.asarray(dev, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(np.abs(ref).max(), 1e-30)
    rel = np.linalg.norm(dev - ref) / max(np.linalg.norm(ref), 1e-30)
    worst = np.abs(dev - ref).max() / scale
    print(f"{what}: rel frob {rel:.2e}, max/scale {worst:.2e}", flush=True)
    assert rel < 1e-3, (what, rel)
    assert worst < 2.0 ** -6, (what, worst)


@pytest.mark.parametrize("E,nin,nh,nout,B", [(3, 37, 64, 3, 77), (2, 129, 96, 3, 32), (1, 5, 32, 1, 1)])
def test_forward_matches_oracle(E, nin, nh, nout, B):
    sur = _cuda()
    print(f"forward E={E} nin={nin} nh={nh} nout={nout} B={B}", flush=True)
    M = _members(E, nin, nh, nout, seed=10 + E)
    X, _ = _data(B, nin, nout, seed=20 + B)
    s = sur.Surrogate(M, nin, nh, nout, max_batch=max(B, 64))
    Y = s.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    for e in range(E):
        ref, _ = mo.forward(M[e], X.astype(np.float64))
        _close(Y[e], ref, f"Y member {e}")
    s.close()


@pytest.mark.parametrize("E,nin,nh,nout,B", [(3, 37, 64, 3, 77), (5, 129, 256, 3, 300), (2, 129, 128, 3, 1500)])
def test_gradients_and_loss_match_oracle(E, nin, nh, nout, B):
    """The last case has batch >= 1024: the weight gradients are summed over
    three k-chunks (512, 512, 480 rows)."""
    sur = _cuda()
    print(f"grads E={E} nin={nin} nh={nh} nout={nout} B={B}", flush=True)
    M = _members(E, nin, nh, nout, seed=30 + E)
    X, T = _data(B, nin, nout, seed=40 + B)
    s = sur.Surrogate(M, nin, nh, nout, max_batch=max(512, B))
    loss = torch.zeros(E, dtype=torch.float32, device="cuda")
    s.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), 0.0, loss)
    G = s.get_grads()
    L = loss.cpu().numpy()
    W = s.get_weights()
    for e in range(E):
        lo, go, _ = mo.loss_and_grads(M[e], X.astype(np.float64), T.astype(np.float64))
        assert abs(L[e] - lo) < 1e-3 * lo, (e, L[e], lo)
        for k in mo_layers():
            _close(G[e][k], go[k], f"grad {k} member {e}")
            # lr = 0 leaves the masters untouched
            assert np.array_equal(W[e][k].astype(np.float64), M[e][k]), k
    s.close()


def mo_layers():
    return ("W1", "b1", "W2", "b2", "W3", "b3")


def test_adam_update_matches_closed_form_on_device_gradients():
    """Two steps: the first step's update from the device's own gradients must
    equal Adam's first-step closed form, the second the recursion, to FP32
    rounding."""
    sur = _cuda()
    E, nin, nh, nout, B = 2, 40, 64, 3, 96
    M = _members(E, nin, nh, nout, seed=5)
    X, T = _data(B, nin, nout, seed=6)
    s = sur.Surrogate(M, nin, nh, nout, max_batch=B)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    lr = 1e-3
    ref = [{k: v.copy() for k, v in m.items()} for m in M]
    state = [{} for _ in range(E)]
    for t in (1, 2):
        s.train_step(Xd, Td, lr)
        G = s.get_grads()
        W = s.get_weights()
        for e in range(E):
            g = {k: G[e][k].astype(np.float64) for k in ref[e]}
            mo.adam_step(ref[e], g, state[e], lr, t)
            for k in ref[e]:
                err = np.abs(W[e][k] - ref[e][k]).max()
                assert err < 2e-6 * max(1.0, np.abs(ref[e][k]).max()), (t, e, k, err)
    s.close()


def test_training_reduces_loss_and_tracks_oracle():
    """Twenty Adam steps from the same weights on the same minibatches: the
    device's weight trajectory follows the oracle's (relative to the distance
    travelled) and the loss falls."""
    sur = _cuda()
    E, nin, nh, nout, B = 2, 24, 64, 3, 128
    M = _members(E, nin, nh, nout, seed=7)
    X, T = _data(B, nin, nout, seed=8)
    s = sur.Surrogate(M, nin, nh, nout, max_batch=B)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    lr = 3e-3
    ref = [{k: v.copy() for k, v in m.items()} for m in M]
    state = [{} for _ in range(E)]
    loss = torch.zeros(E, dtype=torch.float32, device="cuda")
    losses = []
    for t in range(1, 21):
        s.train_step(Xd, Td, lr, loss)
        losses.append(loss.cpu().numpy().copy())
        for e in range(E):
            _, g, _ = mo.loss_and_grads(ref[e], X.astype(np.float64), T.astype(np.float64))
            mo.adam_step(ref[e], g, state[e], lr, t)
    W = s.get_weights()
    for e in range(E):
        for k in ("W1", "W2", "W3"):
            moved = np.linalg.norm(ref[e][k] - M[e][k])
            diff = np.linalg.norm(W[e][k] - ref[e][k])
            print(f"member {e} {k}: moved {moved:.3e} diff {diff:.3e}", flush=True)
            assert diff < 0.05 * moved, (e, k, diff, moved)
        assert losses[-1][e] < 0.7 * losses[0][e], (e, losses[0][e], losses[-1][e])
    s.close()


def test_full_size_forward_sampled_rows():
    """Five members 129 -> 256 -> 256 -> 3 at batch 4096; 64 sampled rows
    against the oracle (rows are independent)."""
    sur = _cuda()
    E, nin, nh, nout, B = 5, 129, 256, 3, 4096
    M = _members(E, nin, nh, nout, seed=9)
    X, _ = _data(B, nin, nout, seed=11)
    s = sur.Surrogate(M, nin, nh, nout, max_batch=B)
    Y = s.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    rows = np.random.default_rng(12).choice(B, size=64, replace=False)
    rows[0], rows[1] = 0, B - 1
    for e in range(E):
        ref, _ = mo.forward(M[e], X[rows].astype(np.float64))
        _close(Y[e][rows], ref, f"full-size member {e}")
    s.close()


def test_history_features_and_gate_match_oracle():
    sur = _cuda()
    n, T = 70, 45
    rng = np.random.default_rng(13)
    grads = rng.normal(size=(T, n, 9))
    ring = torch.zeros((n, 32, 4), dtype=torch.float32, device="cuda")
    phi = torch.from_numpy(rng.uniform(0.1, 0.3, size=n).astype(np.float32)).cuda()
    X = torch.zeros((n, 129), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    for t in range(T):
        sur.push_history(ring, torch.from_numpy(grads[t]).cuda(), t, st)
    sur.features(ring, T - 1, phi, X, st)
    hist = grads[:, :, [0, 1, 3, 4]].transpose(1, 0, 2).astype(np.float32)
    ref = mo.features(hist, phi.cpu().numpy())
    assert np.array_equal(X.cpu().numpy(), ref.astype(np.float32))
    # gate: members spread around a common mean, some flagged
    E, B, nout = 5, 1000, 3
    base = rng.normal(size=(B, nout))
    Y = (base[None] + rng.normal(size=(E, B, nout)) * rng.uniform(0, 0.2, size=(1, B, 1))).astype(np.float32)
    mean = torch.zeros((B, nout), dtype=torch.float32, device="cuda")
    flag = torch.zeros(B, dtype=torch.int32, device="cuda")
    sur.gate(torch.from_numpy(Y).cuda(), 0.05, 0.1, mean, flag, st)
    mu, fl, ratio = mo.gate(Y.astype(np.float64), 0.05, 0.1)
    assert np.abs(mean.cpu().numpy() - mu).max() < 1e-5 * np.abs(mu).max()
    got = flag.cpu().numpy().astype(bool)
    decided = np.abs(ratio - 1.0) > 1e-4
    assert np.array_equal(got[decided], fl[decided])
    assert 0.1 < fl.mean() < 0.9


def test_targets_blend_and_history_gradient_match_oracle():
    sur = _cuda()
    st = torch.cuda.current_stream()
    rng = np.random.default_rng(15)
    n = 300
    sigma = rng.normal(size=(n, 6))
    T = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    sur.targets(torch.from_numpy(sigma).cuda(), 0.5, T, st)
    assert np.allclose(T.cpu().numpy(), mo.targets(sigma, 0.5), rtol=1e-6, atol=1e-6)
    mean = rng.normal(size=(n, 3)).astype(np.float32)
    use = (rng.uniform(size=n) < 0.3).astype(np.uint32)
    out = torch.zeros((n, 6), dtype=torch.float64, device="cuda")
    sur.blend(torch.from_numpy(mean).cuda(), torch.from_numpy(use.astype(np.int32)).cuda(),
              torch.from_numpy(sigma).cuda(), 1.5, out, st)
    assert np.allclose(out.cpu().numpy(), mo.blend(mean.astype(np.float64), use, sigma, 1.5), rtol=1e-12, atol=1e-12)
    # the ring gives back the traceless in-plane gradient it was fed
    ring = torch.zeros((n, 32, 4), dtype=torch.float32, device="cuda")
    a, b, c = (rng.normal(size=n) * 0.1 for _ in range(3))
    L = np.zeros((n, 9))
    L[:, 0], L[:, 1], L[:, 3], L[:, 4] = a, b, c, -a
    sur.push_history(ring, torch.from_numpy(L).cuda(), 40, st, scale=20.0)
    back = torch.zeros((n, 9), dtype=torch.float64, device="cuda")
    sur.history_gradient(ring, 40, back, st, inv_scale=1.0 / 20.0)
    assert np.allclose(back.cpu().numpy(), L, rtol=1e-6, atol=1e-9)


def test_augment_matches_oracle():
    sur = _cuda()
    st = torch.cuda.current_stream()
    rng = np.random.default_rng(17)
    n = 333
    X = rng.normal(size=(n, 129)).astype(np.float32)
    T = rng.normal(size=(n, 3)).astype(np.float32)
    th = rng.uniform(0, 2 * np.pi, size=n).astype(np.float32)
    mir = (rng.uniform(size=n) < 0.5).astype(np.int32)
    Xd, Td = torch.from_numpy(X.copy()).cuda(), torch.from_numpy(T.copy()).cuda()
    sur.augment(Xd, Td, torch.from_numpy(th).cuda(), torch.from_numpy(mir).cuda(), st)
    Xo, To = mo.augment(X.astype(np.float64), T.astype(np.float64), th.astype(np.float64), mir.astype(bool))
    assert np.abs(Xd.cpu().numpy() - Xo).max() < 1e-5 * np.abs(Xo).max()
    assert np.abs(Td.cpu().numpy() - To).max() < 1e-5 * np.abs(To).max()
