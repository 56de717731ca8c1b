"""Python binding of the SPH macro engine and of the coupled exchange
interval (include/lhmm.h: lhmm_sph_*, lhmm_couple_step).  Argument
marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import LhmmSphParams, check, lib
from .micro import Micro

SPH_KEYS = ("rho0", "eta", "zeta", "c", "theta", "F", "h", "dt", "mass", "Lx", "Ly", "lambda_star", "alpha")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Sph:
    """2-D periodic SPH engine on the current GPU."""

    def __init__(self, params: dict, r0: np.ndarray, v0: np.ndarray, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the SPH engine needs a ROCm GPU")
        self._torch = torch
        p = LhmmSphParams(**{k: float(params[k]) for k in SPH_KEYS}, n_fixed=int(params.get("n_fixed", 0)),
                          force_mode=int(params.get("force_mode", 0)), kernel=int(params.get("kernel", 0)),
                          micro_dim=int(params.get("micro_dim", 3)))
        self.n_fixed = int(params.get("n_fixed", 0))
        r0 = np.ascontiguousarray(r0, dtype=np.float64).reshape(-1, 2)
        v0 = np.ascontiguousarray(v0, dtype=np.float64).reshape(-1, 2)
        self.n = r0.shape[0]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        check(lib().lhmm_sph_create(C.byref(p), self.n, _dptr(r0), _dptr(v0), C.c_void_p(self.stream.cuda_stream),
                                    C.byref(h)))
        self._h = h

    def step(self, sigma=None, gradL=None):
        """One velocity-Verlet step; sigma: cuda float64 (n, 6) micro stresses or
        None; gradL: cuda float64 (n, 9) output or None."""
        for t, k in ((sigma, 6), (gradL, 9)):
            if t is not None and (t.dtype != self._torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != k * self.n):
                raise ValueError("stress/gradient buffers must be contiguous cuda float64 of n x 6 / n x 9")
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_sph_step(self._h, C.c_void_p(0 if sigma is None else sigma.data_ptr()),
                                      C.c_void_p(0 if gradL is None else gradL.data_ptr())))

    def get_state(self):
        r = np.zeros((self.n, 2))
        v = np.zeros((self.n, 2))
        d = np.zeros(self.n)
        check(lib().lhmm_sph_get_state(self._h, _dptr(r), _dptr(v), _dptr(d)))
        return r, v, d

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().lhmm_sph_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Coupled:
    """One micro-box per SPH particle; step() is one exchange interval."""

    def __init__(self, sph: Sph, micro: Micro):
        if micro.n_boxes != sph.n - sph.n_fixed:
            raise ValueError("one micro-box per mobile SPH particle is required")
        self.sph, self.micro = sph, micro

    def step(self, k_micro: int, m_bar: int = 1):
        """One exchange interval: m_bar SPH steps, then k_micro micro steps."""
        with self.sph._torch.cuda.stream(self.sph.stream):
            check(lib().lhmm_couple_step(self.sph._h, self.micro._h, int(m_bar), int(k_micro)))

    def coupling_state(self):
        """Host copies of the stored micro stresses (n, 6) and gradients (n, 3, 3)."""
        sig = np.zeros((self.sph.n, 6))
        grad = np.zeros((self.sph.n, 9))
        check(lib().lhmm_sph_coupling_state(self.sph._h, _dptr(sig), _dptr(grad)))
        return sig, grad.reshape(-1, 3, 3)


class Hybrid:
    """The LHMM macro step with the surrogate in the loop (lhmm_hybrid_*).
    mode: "surrogate" or "dpd"; the engines must share one stream and the
    micro engine must be equilibrated."""

    def __init__(self, sph: Sph, micro: Micro, sur=None, phi=None, mode="surrogate", k_micro=50, hold=10,
                 replay=31, threshold=0.05, floor=1.0, grad_scale=1.0, stress_scale=1.0, max_grad=0.0,
                 warm_frac=0.0):
        from ._lib import HYBRID_DPD, HYBRID_SURROGATE, LhmmHybridParams

        p = LhmmHybridParams(mode={"surrogate": HYBRID_SURROGATE, "dpd": HYBRID_DPD}[mode], k_micro=int(k_micro),
                             hold=int(hold), replay=int(replay), threshold=float(threshold), floor=float(floor),
                             grad_scale=float(grad_scale), stress_scale=float(stress_scale),
                             max_grad=float(max_grad), warm_frac=float(warm_frac))
        n_mobile = micro.n_boxes
        phi = np.ascontiguousarray(np.zeros(n_mobile) if phi is None else phi, dtype=np.float32)
        if phi.size != n_mobile:
            raise ValueError("phi needs one value per micro-domain")
        h = C.c_void_p()
        check(lib().lhmm_hybrid_create(C.byref(p), sph._h, micro._h, None if sur is None else sur._h,
                                       phi.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self._h = h
        self.n, self.n_mobile = sph.n, n_mobile
        self._keep = (sph, micro, sur)

    def step(self) -> dict:
        from ._lib import LhmmHybridStats

        st = LhmmHybridStats()
        check(lib().lhmm_hybrid_step(self._h, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in LhmmHybridStats._fields_}

    def state(self):
        sig = np.zeros((self.n, 6))
        on = np.zeros(self.n_mobile, dtype=np.uint32)
        check(lib().lhmm_hybrid_state(self._h, _dptr(sig), on.ctypes.data_as(C.POINTER(C.c_uint32))))
        return sig, on

    def mean_stress(self, reset: bool = False):
        """Mean of the stresses handed to SPH since creation or the last reset (n, 6)."""
        out = np.zeros((self.n, 6))
        check(lib().lhmm_hybrid_mean_stress(self._h, _dptr(out), 1 if reset else 0))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().lhmm_hybrid_destroy(self._h))
            self._h = C.c_void_p()
