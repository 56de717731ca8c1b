"""Python binding of the micro-DPD engine (include/lhmm.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch provides device memory and the caller's stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import LhmmBox, LhmmParams, check, lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Micro:
    """A batch of persistent micro-boxes on the current GPU.

    params: dict with a, gamma, sigma, kBT, mass, rc, dt, H, R0, seed,
    chain_len.  boxes: sequence of (n_particles, n_chains, h0 3x3) or
    (n_particles, n_chains, h0, rng_id); rng_id defaults to the position.
    precision: "fp32" or "fp64".
    """

    def __init__(self, params: dict, boxes: Sequence, precision: str = "fp32", graphs: bool = True,
                 stream=None, components: bool = False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the micro-DPD engine needs a ROCm GPU")
        self._torch = torch
        p = LhmmParams()
        for k in ("a", "gamma", "sigma", "kBT", "mass", "rc", "dt", "H", "R0"):
            setattr(p, k, float(params[k]))
        p.seed = int(params["seed"]) & ((1 << 64) - 1)
        p.chain_len = int(params["chain_len"])
        p.precision = {"fp32": _lib.FP32, "fp64": _lib.FP64}[precision]
        p.flags = (0 if graphs else _lib.OPT_NO_GRAPH) | (_lib.OPT_COMPONENTS if components else 0)
        arr = (LhmmBox * len(boxes))()
        for k, spec in enumerate(boxes):
            n, nch, h0 = spec[0], spec[1], spec[2]
            arr[k].n_particles = int(n)
            arr[k].n_chains = int(nch)
            arr[k].rng_id = int(spec[3]) if len(spec) > 3 else k
            arr[k].reserved = 0
            h = np.asarray(h0, dtype=np.float64).reshape(9)
            for q in range(9):
                arr[k].h0[q] = float(h[q])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = C.c_void_p()
        check(lib().lhmm_micro_create(C.byref(p), arr, len(boxes), C.c_void_p(stream.cuda_stream),
                                      C.byref(handle)))
        self._h = handle
        self.n_boxes = len(boxes)
        self.n_total = int(sum(int(b[0]) for b in boxes))
        self.params = dict(params)
        self.precision = precision

    # -- state ---------------------------------------------------------------
    def set_state(self, s: np.ndarray, c: np.ndarray, h: Optional[np.ndarray] = None, step: int = 0,
                  f: Optional[np.ndarray] = None):
        """Load positions s, velocities c (n_total x 3), optionally cells h and
        the carried forces f (for an exact resume; None = recompute)."""
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(self.n_total, 3)
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.n_total, 3)
        ff = None if f is None else np.ascontiguousarray(f, dtype=np.float64).reshape(self.n_total, 3)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64).reshape(self.n_boxes, 9)
        check(lib().lhmm_micro_set_state(self._h, _dptr(s), _dptr(c), None if ff is None else _dptr(ff),
                                         None if hh is None else _dptr(hh), int(step)))

    def get_state(self, with_forces: bool = False):
        """(s, c, h (n_boxes, 3, 3), step[, f])."""
        s = np.zeros((self.n_total, 3))
        c = np.zeros((self.n_total, 3))
        f = np.zeros((self.n_total, 3))
        h = np.zeros((self.n_boxes, 9))
        st = C.c_uint64()
        check(lib().lhmm_micro_get_state(self._h, _dptr(s), _dptr(c), _dptr(f), _dptr(h), C.byref(st)))
        if with_forces:
            return s, c, h.reshape(self.n_boxes, 3, 3), int(st.value), f
        return s, c, h.reshape(self.n_boxes, 3, 3), int(st.value)

    # -- hot path ------------------------------------------------------------
    def step(self, gradL, n_steps: int, out=None):
        """gradL: cuda float64 tensor (n_boxes, 3, 3) or (n_boxes, 9); returns
        the mean stress over the steps as a cuda float64 tensor (n_boxes, 6)."""
        torch = self._torch
        g = gradL.reshape(self.n_boxes, 9)
        if g.dtype != torch.float64 or not g.is_cuda or not g.is_contiguous():
            raise ValueError("gradL must be a contiguous cuda float64 tensor")
        if out is None:
            out = torch.empty((self.n_boxes, 6), dtype=torch.float64, device=g.device)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != 6 * self.n_boxes:
            raise ValueError("out must be a contiguous cuda float64 tensor of n_boxes x 6")
        with torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_step(self._h, C.c_void_p(g.data_ptr()), int(n_steps),
                                        C.c_void_p(out.data_ptr())))
        return out

    def step_subset(self, gradL, n_steps: int, boxes, out=None):
        """Advance only the listed boxes (strictly increasing indices); rows of
        the other boxes in the returned stress are zero."""
        torch = self._torch
        g = gradL.reshape(self.n_boxes, 9)
        if g.dtype != torch.float64 or not g.is_cuda or not g.is_contiguous():
            raise ValueError("gradL must be a contiguous cuda float64 tensor")
        sel = np.ascontiguousarray(boxes, dtype=np.int32)
        if out is None:
            out = torch.empty((self.n_boxes, 6), dtype=torch.float64, device=g.device)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != 6 * self.n_boxes:
            raise ValueError("out must be a contiguous cuda float64 tensor of n_boxes x 6")
        with torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_step_subset(self._h, C.c_void_p(g.data_ptr()), int(n_steps),
                                               C.c_void_p(out.data_ptr()),
                                               sel.ctypes.data_as(C.POINTER(C.c_int32)), int(sel.size)))
        return out

    def config(self) -> dict:
        c = _lib.LhmmMicroConfig()
        check(lib().lhmm_micro_get_config(self._h, C.byref(c)))
        return {k: int(getattr(c, k)) for k, _ in _lib.LhmmMicroConfig._fields_}

    def set_config(self, **kw):
        cur = self.config()
        cur.update({k: int(v) for k, v in kw.items()})
        c = _lib.LhmmMicroConfig(**cur)
        check(lib().lhmm_micro_set_config(self._h, C.byref(c)))

    def autotune(self, gradL, trial_steps: int = 20):
        """Time launch configurations on the loaded boxes and keep the best
        (the state is unchanged).  Returns (config dict, ms per step)."""
        g = gradL.reshape(self.n_boxes, 9)
        c = _lib.LhmmMicroConfig()
        ms = C.c_double()
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_autotune(self._h, C.c_void_p(g.data_ptr()), int(trial_steps), C.byref(c),
                                            C.byref(ms)))
        return {k: int(getattr(c, k)) for k, _ in _lib.LhmmMicroConfig._fields_}, float(ms.value)

    def snapshot(self):
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_snapshot(self._h))

    def restore(self, boxes):
        sel = np.ascontiguousarray(boxes, dtype=np.int32)
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_restore(self._h, sel.ctypes.data_as(C.POINTER(C.c_int32)), int(sel.size)))

    def time_kernels(self, gradL, n_steps: int) -> dict:
        """Advance n_steps eagerly with HIP events around every kernel on the
        engine's stream; returns {kernel name: mean ms per launch}."""
        g = gradL.reshape(self.n_boxes, 9)
        if g.dtype != self._torch.float64 or not g.is_cuda or not g.is_contiguous():
            raise ValueError("gradL must be a contiguous cuda float64 tensor")
        avg = np.zeros(len(_lib.KERNEL_NAMES))
        with self._torch.cuda.stream(self.stream):
            check(lib().lhmm_micro_time(self._h, C.c_void_p(g.data_ptr()), int(n_steps), _dptr(avg), None))
        return dict(zip(_lib.KERNEL_NAMES, avg.tolist()))

    # -- diagnostics ----------------------------------------------------------
    def forces(self, gradL: np.ndarray):
        g = np.ascontiguousarray(gradL, dtype=np.float64).reshape(self.n_boxes, 9)
        f = np.zeros((self.n_total, 3))
        vir = np.zeros((self.n_boxes, 12))
        check(lib().lhmm_micro_forces(self._h, _dptr(g), _dptr(f), _dptr(vir)))
        return f, vir.reshape(self.n_boxes, 2, 6)

    def stress_parts(self):
        out = np.zeros((self.n_boxes, 3, 6))
        check(lib().lhmm_micro_stress_parts(self._h, _dptr(out)))
        return out

    def pair_counts(self):
        out = np.zeros(self.n_boxes, dtype=np.uint64)
        check(lib().lhmm_micro_pair_counts(self._h, out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out

    def pair_total(self):
        """Unordered pairs within the cutoff over every step since create, per box."""
        out = np.zeros(self.n_boxes, dtype=np.uint64)
        check(lib().lhmm_micro_pair_total(self._h, out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out

    def components(self):
        """(n_boxes, 5, 6) mean stress of the last step call by part: kinetic,
        conservative, dissipative, random, FENE (engine created with components=True)."""
        out = np.zeros((self.n_boxes, 5, 6))
        check(lib().lhmm_micro_components(self._h, _dptr(out)))
        return out

    def set_afbc(self, regions, zeta: float = 10.0):
        """Boundary regions per box: regions (n_boxes, 2) of (core half-width,
        ring outer half-width), (0, 0) for a plain box; zeta: the ring's
        relaxation rate toward the imposed field (lhmm_micro_set_afbc)."""
        r = np.ascontiguousarray(regions, dtype=np.float64).reshape(self.n_boxes, 2)
        check(lib().lhmm_micro_set_afbc(self._h, _dptr(r), float(zeta)))

    def prepare(self, n_steps: int):
        """Capture the graphs a step call of n_steps will replay, without stepping."""
        check(lib().lhmm_micro_prepare(self._h, int(n_steps)))

    def flags(self, clear: bool = False):
        out = np.zeros(self.n_boxes, dtype=np.uint32)
        check(lib().lhmm_micro_flags(self._h, out.ctypes.data_as(C.POINTER(C.c_uint32)), 1 if clear else 0))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().lhmm_micro_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def box_cell(L, edge: float, t_run: float, min_width: float = 3.5):
    """Initial cell for a box under the constant in-plane gradient L over a
    run of t_run time units (lhmm_box_cell): (h (3, 3), kind) with kind
    "cubic", "kr" (Kraynik-Reinelt aligned) or "rotated"."""
    Lv = np.ascontiguousarray(L, dtype=np.float64).reshape(9)
    h = np.zeros(9)
    kind = C.c_int32(-1)
    check(lib().lhmm_box_cell(_dptr(Lv), float(edge), float(t_run), float(min_width), _dptr(h), C.byref(kind)))
    return h.reshape(3, 3), _lib.CELL_KINDS[kind.value]


def from_workload(wl, precision: str = "fp32", graphs: bool = True, rng_ids=None, components: bool = False) -> Micro:
    """Engine holding every box of an ``inputs.Workload`` with its initial state loaded."""
    ids = range(len(wl.boxes)) if rng_ids is None else rng_ids
    boxes = [(b.N, b.n_chains, b.h, k) for b, k in zip(wl.boxes, ids)]
    m = Micro(wl.params, boxes, precision=precision, graphs=graphs, components=components)
    s = np.concatenate([b.s for b in wl.boxes])
    c = np.concatenate([b.c for b in wl.boxes])
    h = np.stack([b.h.reshape(9) for b in wl.boxes])
    m.set_state(s, c, h, 0)
    return m
