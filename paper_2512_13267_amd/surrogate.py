"""Python binding of the stress surrogate (include/lhmm.h: lhmm_sur_*).
Argument marshalling only: every step runs in the library's kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import SUR_FEATURES, SUR_HIST, LhmmSurParams, check, lib

LAYERS = ("W1", "b1", "W2", "b2", "W3", "b3")


def layer_shapes(n_in: int, n_hidden: int, n_out: int):
    return {"W1": (n_in, n_hidden), "b1": (n_hidden,), "W2": (n_hidden, n_hidden), "b2": (n_hidden,),
            "W3": (n_hidden, n_out), "b3": (n_out,)}


def pack(members, n_in, n_hidden, n_out) -> np.ndarray:
    """List of per-member dicts of arrays -> the packed FP32 host layout."""
    shapes = layer_shapes(n_in, n_hidden, n_out)
    parts = []
    for m in members:
        for k in LAYERS:
            a = np.asarray(m[k], dtype=np.float32)
            if a.shape != shapes[k]:
                raise ValueError(f"{k}: shape {a.shape}, expected {shapes[k]}")
            parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unpack(flat: np.ndarray, n_members, n_in, n_hidden, n_out):
    shapes = layer_shapes(n_in, n_hidden, n_out)
    out, o = [], 0
    for _ in range(n_members):
        m = {}
        for k in LAYERS:
            n = int(np.prod(shapes[k]))
            m[k] = flat[o:o + n].reshape(shapes[k]).copy()
            o += n
        out.append(m)
    return out


def init_members(n_members, n_in, n_hidden, n_out, seed):
    """He-style random initialisation, one generator stream per member."""
    rng = np.random.default_rng(seed)
    members = []
    for _ in range(n_members):
        members.append({
            "W1": rng.normal(scale=np.sqrt(2.0 / n_in), size=(n_in, n_hidden)), "b1": np.zeros(n_hidden),
            "W2": rng.normal(scale=np.sqrt(2.0 / n_hidden), size=(n_hidden, n_hidden)), "b2": np.zeros(n_hidden),
            "W3": rng.normal(scale=np.sqrt(1.0 / n_hidden), size=(n_hidden, n_out)), "b3": np.zeros(n_out)})
    return members


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Surrogate:
    """Ensemble of MLPs on the current GPU (BF16 matrix cores, FP32 masters)."""

    def __init__(self, members, n_in, n_hidden, n_out, max_batch, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate engine needs a ROCm GPU")
        self._torch = torch
        self.E, self.n_in, self.n_hidden, self.n_out, self.max_batch = len(members), n_in, n_hidden, n_out, max_batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = LhmmSurParams(self.E, n_in, n_hidden, n_out, max_batch)
        w = pack(members, n_in, n_hidden, n_out)
        h = C.c_void_p()
        check(lib().lhmm_sur_create(C.byref(p), _fptr(w), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def _dev(self, t, cols, name):
        torch = self._torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"{name} must be a contiguous cuda float32 (B, {cols}) tensor")
        return C.c_void_p(t.data_ptr())

    def set_weights(self, members):
        w = pack(members, self.n_in, self.n_hidden, self.n_out)
        check(lib().lhmm_sur_set_weights(self._h, _fptr(w)))

    def get_weights(self):
        n = self.E * sum(int(np.prod(s)) for s in layer_shapes(self.n_in, self.n_hidden, self.n_out).values())
        w = np.zeros(n, dtype=np.float32)
        check(lib().lhmm_sur_get_weights(self._h, _fptr(w)))
        return unpack(w, self.E, self.n_in, self.n_hidden, self.n_out)

    def get_grads(self):
        """Gradients of the last train_step (per-member dicts, FP32)."""
        n = self.E * sum(int(np.prod(s)) for s in layer_shapes(self.n_in, self.n_hidden, self.n_out).values())
        g = np.zeros(n, dtype=np.float32)
        check(lib().lhmm_sur_get_grads(self._h, _fptr(g)))
        return unpack(g, self.E, self.n_in, self.n_hidden, self.n_out)

    def train_step(self, X, T, lr, loss=None):
        """One Adam step of every member on (X, T); loss: optional cuda float32
        (E,) receiving each member's MSE before the step."""
        B = X.shape[0]
        if T.shape[0] != B:
            raise ValueError("X and T must have the same number of rows")
        lp = C.c_void_p(0)
        if loss is not None:
            if loss.dtype != self._torch.float32 or not loss.is_cuda or loss.numel() != self.E:
                raise ValueError("loss must be cuda float32 with n_members entries")
            lp = C.c_void_p(loss.data_ptr())
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_sur_train_step(self._h, self._dev(X, self.n_in, "X"), self._dev(T, self.n_out, "T"), B,
                                            float(lr), lp))

    def forward(self, X, out=None):
        """Predictions (E, B, n_out) cuda float32."""
        B = X.shape[0]
        if out is None:
            out = self._torch.empty((self.E, B, self.n_out), dtype=self._torch.float32, device=X.device)
        if out.dtype != self._torch.float32 or not out.is_contiguous() or out.numel() != self.E * B * self.n_out:
            raise ValueError("out must be contiguous cuda float32 of E x B x n_out")
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_sur_forward(self._h, self._dev(X, self.n_in, "X"), B, C.c_void_p(out.data_ptr())))
        return out

    def forward_static(self, X, out):
        """As forward, through the entry point that allocates nothing (its
        activations live in the library's static device scratch); out is the
        caller's (E, B, n_out) cuda float32 tensor."""
        B = X.shape[0]
        if out.dtype != self._torch.float32 or not out.is_contiguous() or out.numel() != self.E * B * self.n_out:
            raise ValueError("out must be contiguous cuda float32 of E x B x n_out")
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_sur_forward_static(self._h, self._dev(X, self.n_in, "X"), B,
                                                C.c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().lhmm_sur_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def push_history(ring, gradL, t, stream, scale=1.0):
    """ring: cuda float32 (n, SUR_HIST, 4); gradL: cuda float64 (>= n rows of 9)."""
    n = ring.shape[0]
    if ring.shape[1:] != (SUR_HIST, 4) or gradL.numel() < 9 * n:
        raise ValueError("ring must be (n, 32, 4) and gradL (n, 9)")
    check(lib().lhmm_sur_push_history(C.c_void_p(ring.data_ptr()), n, C.c_void_p(gradL.data_ptr()), int(t),
                                      float(scale), C.c_void_p(stream.cuda_stream)))


def history_gradient(ring, t, gradL, stream, inv_scale=1.0):
    n = ring.shape[0]
    if gradL.numel() < 9 * n or gradL.dtype.itemsize != 8:
        raise ValueError("gradL must hold n x 9 float64")
    check(lib().lhmm_sur_history_gradient(C.c_void_p(ring.data_ptr()), n, int(t), float(inv_scale),
                                          C.c_void_p(gradL.data_ptr()), C.c_void_p(stream.cuda_stream)))


def augment(X, T, theta, mirror, stream):
    """In-place symmetry images of rows of X (n, 129) and T (n, 3), cuda float32."""
    n = X.shape[0]
    if X.shape != (n, SUR_FEATURES) or T.shape != (n, 3) or theta.numel() != n or mirror.numel() != n:
        raise ValueError("X (n, 129), T (n, 3), theta (n,), mirror (n,)")
    check(lib().lhmm_sur_augment(C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                 C.c_void_p(theta.data_ptr()), C.c_void_p(mirror.data_ptr()),
                                 C.c_void_p(stream.cuda_stream)))


def targets(sigma, inv_scale, T, stream):
    """sigma: cuda float64 (n, 6) -> T cuda float32 (n, 3)."""
    n = T.shape[0]
    if sigma.numel() < 6 * n or T.shape != (n, 3):
        raise ValueError("sigma must hold n x 6 and T be (n, 3)")
    check(lib().lhmm_sur_targets(C.c_void_p(sigma.data_ptr()), n, float(inv_scale), C.c_void_p(T.data_ptr()),
                                 C.c_void_p(stream.cuda_stream)))


def blend(mean, use_dpd, sigma_dpd, scale, out, stream):
    n = mean.shape[0]
    check(lib().lhmm_sur_blend(C.c_void_p(mean.data_ptr()),
                               C.c_void_p(0 if use_dpd is None else use_dpd.data_ptr()),
                               C.c_void_p(0 if sigma_dpd is None else sigma_dpd.data_ptr()), n, float(scale),
                               C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)))


def features(ring, t, phi, X, stream):
    """X: cuda float32 (n, SUR_FEATURES) from the ring after sample t."""
    n = ring.shape[0]
    if X.shape != (n, SUR_FEATURES) or phi.numel() != n:
        raise ValueError("X must be (n, 129) and phi (n,)")
    check(lib().lhmm_sur_features(C.c_void_p(ring.data_ptr()), n, int(t), C.c_void_p(phi.data_ptr()),
                                  C.c_void_p(X.data_ptr()), C.c_void_p(stream.cuda_stream)))


def gate(Y, threshold, floor, mean, flag, stream):
    """Y: (E, B, n_out) float32; mean (B, n_out) float32; flag (B,) int32."""
    E, B, n_out = Y.shape
    if mean.shape != (B, n_out) or flag.numel() != B or flag.element_size() != 4:
        raise ValueError("mean must be (B, n_out) and flag (B,) 32-bit")
    check(lib().lhmm_sur_gate(C.c_void_p(Y.data_ptr()), E, B, n_out, float(threshold), float(floor),
                              C.c_void_p(mean.data_ptr()), C.c_void_p(flag.data_ptr()),
                              C.c_void_p(stream.cuda_stream)))


TRAINED = __import__("os").path.join(__import__("os").path.dirname(__file__), "weights", "surrogate_e5_h256.npz")
# the training set of the packaged weights: train.generate(n_boxes, n_macro, seed_k) with the default
# gradient amplitudes and correlation time (train.input_quantile reproduces its inputs)
TRAINED_DATA = {"n_boxes": 8192, "n_macro": 520, "seed_k": 3}


def load_trained(path: str = TRAINED):
    """Members (list of dicts), hidden width, grad_scale, stress_scale of a
    weights file written by the training pipeline."""
    z = np.load(path, allow_pickle=False)
    E = int(z["n_members"])
    members = [{k: z[f"m{e}_{k}"].astype(np.float64) for k in LAYERS} for e in range(E)]
    return members, int(z["n_hidden"]), float(z["grad_scale"]), float(z["stress_scale"])
