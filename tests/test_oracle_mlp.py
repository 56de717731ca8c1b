"""Pins of the surrogate oracle (oracle/mlp_oracle.py).

* bfloat16 rounding against torch's float32 -> bfloat16 conversion (a
  library routine) and its ties-to-even rule;
* gradients of the exact (unrounded) float64 network against central finite
  differences of its loss;
* with BF16 rounding the analytic gradients stay within the BF16 error bound
  of the exact ones;
* Adam against its closed form for a constant gradient (m_hat = g,
  v_hat = g^2, so every step moves each weight by -lr g/(|g| + eps)).
"""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo


def _params(rng, nin=7, nh=9, nout=3, scale=0.5):
    return {"W1": rng.normal(scale=scale, size=(nin, nh)), "b1": rng.normal(scale=0.1, size=nh),
            "W2": rng.normal(scale=scale, size=(nh, nh)), "b2": rng.normal(scale=0.1, size=nh),
            "W3": rng.normal(scale=scale, size=(nh, nout)), "b3": rng.normal(scale=0.1, size=nout)}


def test_bf16_rounding_matches_library_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [0.0, -0.0, 1.0, -2.5, 65504.0, 1e-30]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mo.bf16(x), ref)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert mo.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mo.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def _exact_loss(params, X, T):
    return float(np.mean((mo.forward_exact(params, X) - T) ** 2))


def _exact_grads(params, X, T):
    """Backward of the float64 network without rounding, same formulas."""
    H0 = X
    Z1 = H0 @ params["W1"] + params["b1"]
    H1 = mo.gelu(Z1)
    Z2 = H1 @ params["W2"] + params["b2"]
    H2 = mo.gelu(Z2)
    Y = H2 @ params["W3"] + params["b3"]
    B, nout = T.shape
    dY = 2 * (Y - T) / (B * nout)
    dZ2 = (dY @ params["W3"].T) * mo.gelu_grad(Z2)
    dZ1 = (dZ2 @ params["W2"].T) * mo.gelu_grad(Z1)
    return {"W3": H2.T @ dY, "b3": dY.sum(0), "W2": H1.T @ dZ2, "b2": dZ2.sum(0), "W1": X.T @ dZ1, "b1": dZ1.sum(0)}


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    P = _params(rng)
    X = rng.normal(size=(11, 7))
    T = rng.normal(size=(11, 3))
    g = _exact_grads(P, X, T)
    eps = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = _exact_loss(P, X, T)
            flat[idx] = old - eps
            lm = _exact_loss(P, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(g[k].reshape(-1)[idx] - fd) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_rounded_gradients_within_bf16_bound():
    rng = np.random.default_rng(2)
    P = _params(rng, nin=16, nh=32, nout=3)
    X = rng.normal(size=(64, 16))
    T = rng.normal(size=(64, 3))
    _, g, _ = mo.loss_and_grads(P, X, T)
    ge = _exact_grads(P, X, T)
    for k in P:
        scale = np.abs(ge[k]).max()
        assert np.abs(g[k] - ge[k]).max() < 0.05 * scale, k


def test_adam_closed_form_constant_gradient():
    rng = np.random.default_rng(3)
    P = {"w": rng.normal(size=(5, 4))}
    g = {"w": rng.normal(size=(5, 4))}
    w0 = P["w"].copy()
    state = {}
    lr = 1e-2
    for t in range(1, 8):
        mo.adam_step(P, g, state, lr, t)
    step = lr * g["w"] / (np.abs(g["w"]) + mo.ADAM_EPS)
    assert np.allclose(P["w"], w0 - 7 * step, rtol=1e-10, atol=1e-12)


def test_gelu_derivative():
    z = np.linspace(-6, 6, 101)
    eps = 1e-6
    fd = (mo.gelu(z + eps) - mo.gelu(z - eps)) / (2 * eps)
    assert np.allclose(mo.gelu_grad(z), fd, atol=1e-8)
    assert mo.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mo.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_gate_special_cases():
    # identical members: zero spread, never flagged, mean = the member
    Y1 = np.tile(np.array([[[1.0, -2.0, 0.5], [0.0, 0.0, 0.0]]]), (5, 1, 1))
    mu, flag, ratio = mo.gate(Y1, 0.05, 0.1)
    assert np.array_equal(mu, Y1[0]) and not flag.any() and np.all(ratio == 0)
    # two members at +-d around m: spread = d exactly (population variance)
    m = np.array([3.0, 4.0, 0.0])
    d = 0.2
    Y2 = np.stack([m + d, m - d])[:, None, :]
    mu, flag, ratio = mo.gate(Y2, 0.05, 0.1)
    assert np.allclose(mu[0], m) and abs(ratio[0] - d / (0.05 * 5.0)) < 1e-12 and not flag[0]
    _, flag, _ = mo.gate(np.stack([m + 0.3, m - 0.3])[:, None, :], 0.05, 0.1)
    assert flag[0]
    # below the floor the denominator is the floor
    Y3 = np.stack([np.full(3, 1e-3), np.full(3, -1e-3)])[:, None, :]
    _, _, ratio = mo.gate(Y3, 0.05, 0.1)
    assert abs(ratio[0] - 1e-3 / (0.05 * 0.1)) < 1e-12


def test_features_order():
    n, T = 3, 40
    hist = np.arange(n * T * 4, dtype=np.float64).reshape(n, T, 4)
    X = mo.features(hist, np.array([0.1, 0.2, 0.3]))
    assert X.shape == (3, 129)
    # first feature = oldest kept sample (index T-32), component xx
    assert X[1, 0] == hist[1, T - 32, 0] and X[1, 127] == hist[1, T - 1, 3] and X[2, 128] == 0.3


def test_targets_and_blend_pins():
    rng = np.random.default_rng(14)
    # an isotropic stress has no deviatoric part
    iso = np.tile(np.array([[2.5, 2.5, 2.5, 0.0, 0.0, 0.0]]), (3, 1))
    assert np.abs(mo.targets(iso)).max() == 0.0
    # simple shear stress: only xy survives
    sh = np.array([[0.0, 0.0, 0.0, 0.7, 0.0, 0.0]])
    assert np.allclose(mo.targets(sh, 2.0), [[0.0, 1.4, 0.0]])
    # a blended surrogate row is traceless and its targets give back the mean
    mean = rng.normal(size=(6, 3))
    out = mo.blend(mean, None, None, 1.7)
    assert np.allclose(out[:, :3].sum(axis=1), 0.0)
    assert np.allclose(mo.targets(out, 1.0 / 1.7), mean)
    # rows flagged for DPD are the micro stress unchanged
    sd = rng.normal(size=(6, 6))
    use = np.array([1, 0, 0, 1, 0, 1])
    out = mo.blend(mean, use, sd, 1.0)
    assert np.array_equal(out[use == 1], sd[use == 1])


def test_augment_group_pins():
    rng = np.random.default_rng(16)
    n = 7
    X = rng.normal(size=(n, 129))
    T = rng.normal(size=(n, 3))
    zero = np.zeros(n)
    none = np.zeros(n, dtype=bool)
    # identity and full turn
    for th in (zero, np.full(n, 2 * math.pi)):
        X1, T1 = mo.augment(X, T, th, none)
        assert np.allclose(X1, X, atol=1e-12) and np.allclose(T1, T, atol=1e-12)
    # two rotations compose; a reflection applied twice is the identity
    a, b = rng.uniform(0, 6.3, n), rng.uniform(0, 6.3, n)
    X2, T2 = mo.augment(*mo.augment(X, T, a, none), b, none)
    X3, T3 = mo.augment(X, T, a + b, none)
    assert np.allclose(X2, X3) and np.allclose(T2, T3)
    Xm, Tm = mo.augment(*mo.augment(X, T, zero, ~none), zero, ~none)
    assert np.allclose(Xm, X) and np.allclose(Tm, T)
    # a quarter turn maps simple shear u_x = g y to u_y = -g x: L_xy -> -L_yx
    Xs = np.zeros((1, 129))
    Xs[0, 1] = 1.0
    Xq, _ = mo.augment(Xs, np.zeros((1, 3)), np.array([math.pi / 2]), np.array([False]))
    assert np.allclose(Xq[0, :4], [0.0, 0.0, -1.0, 0.0], atol=1e-12)
    # invariants: trace and Frobenius norm of every sample and of S; phi kept
    Xr, Tr = mo.augment(X, T, a, rng.uniform(size=n) < 0.5)
    for k in range(32):
        L0, L1 = X[:, 4 * k:4 * k + 4], Xr[:, 4 * k:4 * k + 4]
        assert np.allclose(L0[:, 0] + L0[:, 3], L1[:, 0] + L1[:, 3])
        assert np.allclose((L0 ** 2).sum(1), (L1 ** 2).sum(1))
    assert np.allclose(T[:, 0] + T[:, 2], Tr[:, 0] + Tr[:, 2])
    assert np.allclose(T[:, 0] ** 2 + 2 * T[:, 1] ** 2 + T[:, 2] ** 2, Tr[:, 0] ** 2 + 2 * Tr[:, 1] ** 2 + Tr[:, 2] ** 2)
    assert np.array_equal(Xr[:, 128], X[:, 128])
    # reflection y -> -y flips the sign of every xy / yx component
    Xf, Tf = mo.augment(X, T, zero, ~none)
    assert np.allclose(Xf[:, 1:128:4], -X[:, 1:128:4]) and np.allclose(Tf[:, 1], -T[:, 1])
