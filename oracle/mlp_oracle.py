"""Double-precision oracle of the stress surrogate: an ensemble of MLPs
(inputs -> hidden -> hidden -> outputs, GELU), mean-squared-error loss and
Adam, with the mixed-precision dataflow of the device path written out.

TEST INFRASTRUCTURE ONLY.  Plain numpy in float64.  The device multiplies
BF16 operands with FP32 accumulation; the points where its operands are
rounded to BF16 are part of the method's definition, so this oracle rounds at
the same points (``bf16``, round to nearest even) and computes everything
else in float64:

forward   Z1 = bf(X) bf(W1) + b1,  H1 = gelu(Z1)
          Z2 = bf(H1) bf(W2) + b2, H2 = gelu(Z2)
          Y  = bf(H2) bf(W3) + b3
loss      (1 / (B n_out)) sum (Y - T)^2              (per member)
backward  dY  = 2 (Y - T) / (B n_out)
          dW3 = bf(H2)^T bf(dY),  db3 = sum_b dY
          dZ2 = (bf(dY) bf(W3)^T) * gelu'(Z2),  dW2 = bf(H1)^T bf(dZ2), db2
          dZ1 = (bf(dZ2) bf(W2)^T) * gelu'(Z1), dW1 = bf(X)^T bf(dZ1),  db1
Adam      m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
          w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
with gelu(z) = z Phi(z) (erf form) and gelu'(z) = Phi(z) + z phi(z).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (8-bit mantissa), to nearest, ties to
    even, via the float32 bit pattern; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, X):
    """params: dict W1 (nin x nh), b1, W2 (nh x nh), b2, W3 (nh x nout), b3.
    Returns Y and the cache for backward."""
    Z1 = bf16(X) @ bf16(params["W1"]) + params["b1"]
    H1 = gelu(Z1)
    Z2 = bf16(H1) @ bf16(params["W2"]) + params["b2"]
    H2 = gelu(Z2)
    Y = bf16(H2) @ bf16(params["W3"]) + params["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(params, X, T):
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    B, nout = T.shape
    loss = float(np.mean((Y - T) ** 2))
    dY = 2.0 * (Y - T) / (B * nout)
    g = {}
    g["W3"] = bf16(H2).T @ bf16(dY)
    g["b3"] = dY.sum(axis=0)
    dZ2 = (bf16(dY) @ bf16(params["W3"]).T) * gelu_grad(Z2)
    g["W2"] = bf16(H1).T @ bf16(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (bf16(dZ2) @ bf16(params["W2"]).T) * gelu_grad(Z1)
    g["W1"] = bf16(X).T @ bf16(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return loss, g, Y


def adam_step(params, grads, state, lr, t):
    """In-place Adam (step number t >= 1) on float64 params; state holds m, v."""
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = ADAM_B1 * m + (1.0 - ADAM_B1) * grads[k]
        v[...] = ADAM_B2 * v + (1.0 - ADAM_B2) * grads[k] ** 2
        mh = m / (1.0 - ADAM_B1 ** t)
        vh = v / (1.0 - ADAM_B2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + ADAM_EPS)
    return params


def forward_exact(params, X):
    """The same network without any BF16 rounding (float64 throughout)."""
    H1 = gelu(X @ params["W1"] + params["b1"])
    H2 = gelu(H1 @ params["W2"] + params["b2"])
    return H2 @ params["W3"] + params["b3"]


def features(history, phi):
    """Feature rows of the surrogate: history (n, T, 4) holds each particle's
    gradient samples (L_xx, L_xy, L_yx, L_yy) in time order; the row is the
    last 32 samples, oldest first, flattened, then the polymer fraction."""
    h = np.asarray(history, dtype=np.float64)
    last = h[:, -32:, :].reshape(h.shape[0], -1)
    return np.concatenate([last, np.asarray(phi, dtype=np.float64)[:, None]], axis=1)


def gate(Y, threshold, floor):
    """Ensemble mean and disagreement flag of member predictions Y
    (members, B, n_out): spread = sqrt(mean over outputs of the population
    variance across members); flagged where spread > threshold x
    max(|mean|_2, floor).  Returns (mean, flag, ratio) with ratio = spread /
    (threshold x max(|mean|_2, floor))."""
    Y = np.asarray(Y, dtype=np.float64)
    mu = Y.mean(axis=0)
    var = ((Y - mu) ** 2).mean(axis=0)
    spread = np.sqrt(var.mean(axis=1))
    denom = threshold * np.maximum(np.sqrt((mu ** 2).sum(axis=1)), floor)
    ratio = spread / denom
    return mu, ratio > 1.0, ratio


def targets(sigma, inv_scale=1.0):
    """In-plane deviatoric part (xx - tr/3, xy, yy - tr/3) of micro stresses
    sigma (n, 6) = (xx, yy, zz, xy, xz, yz), times inv_scale: what the
    macro momentum equation takes from a micro-domain (Eq. pip, before the
    factor alpha/lambda*)."""
    s = np.asarray(sigma, dtype=np.float64)
    tr3 = s[:, :3].sum(axis=1) / 3.0
    return np.stack([s[:, 0] - tr3, s[:, 3], s[:, 1] - tr3], axis=1) * inv_scale


def blend(mean, use_dpd, sigma_dpd, scale=1.0):
    """Stress rows for the macro solver: the micro stress where use_dpd,
    else the traceless tensor whose in-plane deviatoric part is scale x mean."""
    m = np.asarray(mean, dtype=np.float64) * scale
    out = np.zeros((m.shape[0], 6))
    out[:, 0], out[:, 1], out[:, 2], out[:, 3] = m[:, 0], m[:, 2], -(m[:, 0] + m[:, 2]), m[:, 1]
    if use_dpd is not None:
        u = np.asarray(use_dpd).astype(bool)
        out[u] = np.asarray(sigma_dpd)[u]
    return out


def augment(X, T, theta, mirror, hist=32):
    """Symmetry images of surrogate samples under the in-plane orthogonal
    group: each row b is reflected (y -> -y) when mirror[b], then rotated
    by theta[b].  Gradient samples transform as L' = Q L Q^T and the stress
    targets as S' = Q S Q^T with S = [[s_xx, s_xy], [s_xy, s_yy]]
    (the micro model is isotropic, so these are samples of the same
    conditional law).  The polymer-fraction column is unchanged."""
    X = np.asarray(X, dtype=np.float64).copy()
    T = np.asarray(T, dtype=np.float64).copy()
    for b in range(X.shape[0]):
        c, s = math.cos(theta[b]), math.sin(theta[b])
        Q = np.array([[c, -s], [s, c]]) @ (np.diag([1.0, -1.0]) if mirror[b] else np.eye(2))
        for k in range(hist):
            L = X[b, 4 * k:4 * k + 4].reshape(2, 2)
            X[b, 4 * k:4 * k + 4] = (Q @ L @ Q.T).reshape(4)
        S = np.array([[T[b, 0], T[b, 1]], [T[b, 1], T[b, 2]]])
        S = Q @ S @ Q.T
        T[b] = [S[0, 0], S[0, 1], S[1, 1]]
    return X, T
