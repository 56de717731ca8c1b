"""ctypes binding of the C oracle (``lhmm_oracle.c``).

Test infrastructure only.  Arrays are numpy float64 / uint32; particle
arrays are N x 3 (row per particle), cells are 3 x 3 row-major with the
lattice vectors as columns (r = h s).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lhmm_oracle.c")
SOURCES = [SRC, os.path.join(HERE, "sph_oracle.c")]
LIB = os.path.join(HERE, "liblhmm_oracle.so")

ERR_BOND = 1
ERR_CELL = 2
ERR_NONFINITE = 4
ERR_ARG = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (double precision, no fast-math, no FMA
    contraction, OpenMP over boxes)."""
    if force or _stale():
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, *SOURCES, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _stale() -> bool:
    return not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SOURCES)


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint32)
        ip = C.POINTER(C.c_int)
        u64p = C.POINTER(C.c_uint64)
        L.oracle_philox4x32_10.argtypes = [up, up, up]
        L.oracle_uniform23.argtypes = [C.c_uint32]
        L.oracle_uniform23.restype = C.c_double
        L.oracle_theta.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_theta.restype = C.c_double
        L.oracle_check_gradient.argtypes = [dp]
        L.oracle_check_gradient.restype = C.c_int
        L.oracle_expL.argtypes = [dp, C.c_double, dp]
        L.oracle_widths.argtypes = [dp, dp]
        L.oracle_reduce_cell.argtypes = [dp, ip]
        L.oracle_reduce_cell.restype = C.c_int
        L.oracle_pairs.argtypes = [C.c_int, dp, dp, C.c_double, C.c_int, ip, dp, C.c_long]
        L.oracle_pairs.restype = C.c_long
        L.oracle_forces.argtypes = [dp, C.c_uint64, C.c_int, C.c_uint32, C.c_int, C.c_int, dp, dp, dp,
                                    dp, C.c_uint32, dp, dp, up, C.c_int, C.POINTER(C.c_longlong)]
        L.oracle_forces.restype = C.c_int
        L.oracle_run_box.argtypes = [dp, C.c_uint64, C.c_int, C.c_uint32, C.c_int, C.c_int, dp, dp, dp,
                                     ip, dp, u64p, dp, C.c_int, dp, dp, dp, up, C.c_int,
                                     C.POINTER(C.c_longlong)]
        L.oracle_run_box.restype = C.c_int
        L.oracle_run_batch.argtypes = [dp, C.c_uint64, C.c_int, C.c_int, ip, ip, up, dp, dp, dp, ip, dp,
                                       u64p, dp, C.c_int, dp, dp, up, C.c_int, C.POINTER(C.c_longlong)]
        L.oracle_run_batch.restype = C.c_int
        L.oracle_max_threads.restype = C.c_int
        L.oracle_afbc_region.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_afbc_region.restype = C.c_int
        L.oracle_core_fraction.argtypes = [dp, dp, C.c_double]
        L.oracle_core_fraction.restype = C.c_double
        L.oracle_run_box_afbc.argtypes = [dp, C.c_uint64, C.c_int, C.c_uint32, C.c_int, C.c_int, dp, dp, dp,
                                          ip, dp, u64p, dp, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp,
                                          up, C.c_int]
        L.oracle_afbc_noise.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.oracle_run_box_afbc.restype = C.c_int
        L.oracle_sph_W.argtypes = [C.c_double, C.c_double, C.c_int]
        L.oracle_sph_W.restype = C.c_double
        L.oracle_sph_F.argtypes = [C.c_double, C.c_double, C.c_int]
        L.oracle_sph_F.restype = C.c_double
        L.oracle_sph_density.argtypes = [dp, C.c_int, dp, dp, dp]
        L.oracle_sph_gradv.argtypes = [dp, C.c_int, dp, dp, dp, dp]
        L.oracle_sph_accel.argtypes = [dp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.oracle_sph_step.argtypes = [dp, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_sph_polymer_stress.argtypes = [dp, C.c_int, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _u64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _f64(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_u(c), _u(k), _u(out))
    return out


def uniform23(x: int) -> float:
    return lib().oracle_uniform23(int(x))


def theta(seed: int, i: int, j: int, step: int, box: int) -> float:
    return lib().oracle_theta(seed, i, j, step, box)


def check_gradient(L) -> bool:
    return bool(lib().oracle_check_gradient(_d(_f64(L, (9,)))))


def expL(L, tau: float):
    E = np.zeros(9)
    lib().oracle_expL(_d(_f64(L, (9,))), float(tau), _d(E))
    return E.reshape(3, 3)


def widths(h):
    w = np.zeros(3)
    lib().oracle_widths(_d(_f64(h, (9,))), _d(w))
    return w


def reduce_cell(h):
    hh = _f64(h, (9,)).copy()
    U = np.zeros(4, dtype=np.int32)
    changed = lib().oracle_reduce_cell(_d(hh), _i(U))
    return hh.reshape(3, 3), U.reshape(2, 2), bool(changed)


def pairs(s, h, rc: float, mode: int):
    """Unordered pairs (i < j) with 0 < r < rc; mode 0 brute force, 1 cell grid."""
    s = _f64(s)
    N = s.shape[0]
    hh = _f64(h, (9,))
    cap = max(16, 40 * N)
    ij = np.zeros(2 * cap, dtype=np.int32)
    d = np.zeros(3 * cap)
    n = lib().oracle_pairs(N, _d(s), _d(hh), float(rc), int(mode), _i(ij), _d(d), cap)
    if n < 0:
        return None, None
    if n > cap:
        raise RuntimeError("pair capacity exceeded")
    return ij[: 2 * n].reshape(n, 2), d[: 3 * n].reshape(n, 3)


def params_vector(p) -> np.ndarray:
    return np.array([p["a"], p["gamma"], p["sigma"], p["kBT"], p["mass"], p["rc"], p["dt"], p["H"], p["R0"]],
                    dtype=np.float64)


def forces(p, seed, chain_len, box, n_chains, s, c, h, L, step, mode=1):
    """Forces (N x 3), virial parts (4 x 6: C, D, R, FENE) and error bits."""
    P = params_vector(p)
    s = _f64(s)
    c = _f64(c)
    N = s.shape[0]
    F = np.zeros((N, 3))
    W = np.zeros(24)
    err = np.zeros(1, dtype=np.uint32)
    lib().oracle_forces(_d(P), int(seed), int(chain_len), int(box), N, int(n_chains), _d(s), _d(c),
                        _d(_f64(h, (9,))), _d(_f64(L, (9,))), int(step), _d(F), _d(W), _u(err), int(mode), None)
    return F, W.reshape(4, 6), int(err[0])


@dataclass
class OracleBox:
    """One micro-box's oracle state."""
    s: np.ndarray
    c: np.ndarray
    h: np.ndarray
    n_chains: int
    box_id: int = 0
    step: int = 0
    F: np.ndarray = field(default=None)
    fvalid: int = 0
    err: int = 0

    def __post_init__(self):
        self.s = _f64(self.s).copy()
        self.c = _f64(self.c).copy()
        self.h = _f64(self.h, (3, 3)).copy()
        if self.F is None:
            self.F = np.zeros_like(self.s)


def run_box(p, seed, chain_len, box: OracleBox, L, nsteps, mode=1, series=False):
    """Advance ``box`` in place; returns (mean stress (6,), parts (5, 6), series or None)."""
    P = params_vector(p)
    N = box.s.shape[0]
    fv = np.array([box.fvalid], dtype=np.int32)
    st = np.array([box.step], dtype=np.uint64)
    err = np.array([box.err], dtype=np.uint32)
    h = box.h.reshape(9).copy()
    mean = np.zeros(6)
    parts = np.zeros(30)
    ser = np.zeros(6 * nsteps) if series else None
    rc = lib().oracle_run_box(_d(P), int(seed), int(chain_len), int(box.box_id), N, int(box.n_chains),
                              _d(box.s), _d(box.c), _d(box.F), _i(fv), _d(h), _u64(st), _d(_f64(L, (9,))),
                              int(nsteps), _d(mean), _d(parts), _d(ser) if series else None, _u(err), int(mode),
                              None)
    box.h = h.reshape(3, 3)
    box.fvalid = int(fv[0])
    box.step = int(st[0])
    box.err = int(err[0])
    if rc != 0:
        raise ValueError("oracle_run_box rejected its arguments (error bits %d)" % box.err)
    return mean, parts.reshape(5, 6), (ser.reshape(nsteps, 6) if series else None)


def run_batch(p, seed, chain_len, boxes, Ls, nsteps, mode=1, count_pairs=False):
    """Advance a list of OracleBox in one OpenMP call; returns (means (B,6),
    parts (B,5,6)) and, with count_pairs, the pairs evaluated per box."""
    P = params_vector(p)
    B = len(boxes)
    off = np.zeros(B + 1, dtype=np.int32)
    for b, bx in enumerate(boxes):
        off[b + 1] = off[b] + bx.s.shape[0]
    s = np.concatenate([bx.s for bx in boxes]) if B else np.zeros((0, 3))
    c = np.concatenate([bx.c for bx in boxes]) if B else np.zeros((0, 3))
    F = np.concatenate([bx.F for bx in boxes]) if B else np.zeros((0, 3))
    s = np.ascontiguousarray(s)
    c = np.ascontiguousarray(c)
    F = np.ascontiguousarray(F)
    nch = np.array([bx.n_chains for bx in boxes], dtype=np.int32)
    ids = np.array([bx.box_id for bx in boxes], dtype=np.uint32)
    fv = np.array([bx.fvalid for bx in boxes], dtype=np.int32)
    h = np.ascontiguousarray(np.stack([bx.h.reshape(9) for bx in boxes])) if B else np.zeros((0, 9))
    st = np.array([bx.step for bx in boxes], dtype=np.uint64)
    err = np.array([bx.err for bx in boxes], dtype=np.uint32)
    Lv = np.ascontiguousarray(_f64(Ls).reshape(B, 9))
    mean = np.zeros((B, 6))
    parts = np.zeros((B, 30))
    npairs = np.zeros(B, dtype=np.int64)
    rc = lib().oracle_run_batch(_d(P), int(seed), int(chain_len), B, _i(off), _i(nch), _u(ids), _d(s), _d(c),
                                _d(F), _i(fv), _d(h), _u64(st), _d(Lv), int(nsteps), _d(mean), _d(parts),
                                _u(err), int(mode), npairs.ctypes.data_as(C.POINTER(C.c_longlong)))
    for b, bx in enumerate(boxes):
        bx.s = s[off[b]:off[b + 1]].copy()
        bx.c = c[off[b]:off[b + 1]].copy()
        bx.F = F[off[b]:off[b + 1]].copy()
        bx.h = h[b].reshape(3, 3).copy()
        bx.fvalid = int(fv[b])
        bx.step = int(st[b])
        bx.err = int(err[b])
    if rc != 0:
        raise ValueError("oracle_run_batch rejected its arguments")
    if count_pairs:
        return mean, parts.reshape(B, 5, 6), npairs
    return mean, parts.reshape(B, 5, 6)


def afbc_region(x: float, y: float, hc: float, hb: float) -> int:
    """0 core, 1 boundary-condition ring, 2 buffer (position relative to the cell centre)."""
    return int(lib().oracle_afbc_region(float(x), float(y), float(hc), float(hb)))


def core_fraction(a, b, hc: float) -> float:
    """Fraction of the in-plane segment a -> b inside the square |x|, |y| <= hc."""
    return float(lib().oracle_core_fraction(_d(_f64(a, (2,)).copy()), _d(_f64(b, (2,)).copy()), float(hc)))


def afbc_noise(seed: int, i: int, half: int, step: int, box: int):
    """The two normals particle i of the ring draws at a half kick."""
    xi = np.zeros(2)
    lib().oracle_afbc_noise(int(seed), int(i), int(half), int(step), int(box), _d(xi))
    return xi


def run_box_afbc(p, seed, chain_len, box: OracleBox, G, hc: float, hb: float, nsteps: int, zeta: float = 10.0,
                 mode=1):
    """Advance a micro-domain with boundary regions in place (fixed cell
    box.h; on the ring hc <= max(|x'|, |y'|) < hb the in-plane velocity
    relaxes toward the imposed field G r' at rate zeta with thermal noise;
    core stress); returns (mean stress (6,), parts (5, 6))."""
    P = params_vector(p)
    N = box.s.shape[0]
    fv = np.array([box.fvalid], dtype=np.int32)
    st = np.array([box.step], dtype=np.uint64)
    err = np.array([box.err], dtype=np.uint32)
    h = box.h.reshape(9).copy()
    mean = np.zeros(6)
    parts = np.zeros(30)
    rc = lib().oracle_run_box_afbc(_d(P), int(seed), int(chain_len), int(box.box_id), N, int(box.n_chains),
                                   _d(box.s), _d(box.c), _d(box.F), _i(fv), _d(h), _u64(st), _d(_f64(G, (9,))),
                                   float(hc), float(hb), float(zeta), int(nsteps), _d(mean), _d(parts), _u(err),
                                   int(mode))
    box.fvalid = int(fv[0])
    box.step = int(st[0])
    box.err = int(err[0])
    if rc != 0:
        raise ValueError("oracle_run_box_afbc rejected its arguments (error bits %d)" % box.err)
    return mean, parts.reshape(5, 6)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------------------
# SPH macro side
# ---------------------------------------------------------------------------

def sph_params_vector(q) -> np.ndarray:
    keys = ["rho0", "eta", "zeta", "c", "theta", "F", "h", "dt", "mass", "Lx", "Ly", "lambda_star", "alpha"]
    vals = [float(q[k]) for k in keys] + [float(q.get("n_fixed", 0)), float(q.get("force_mode", 0)),
                                          float(q.get("kernel", 0)), float(q.get("micro_dim", 3))]
    return np.array(vals, dtype=np.float64)


def sph_W(r, h, kernel=0):
    """kernel 0: quintic spline, 1: Lucy (Eq. lucy_kernel)."""
    return lib().oracle_sph_W(float(r), float(h), int(kernel))


def sph_F(r, h, kernel=0):
    return lib().oracle_sph_F(float(r), float(h), int(kernel))


def sph_density(q, r):
    P = sph_params_vector(q)
    r = _f64(r)
    n = r.shape[0]
    d = np.zeros(n)
    p = np.zeros(n)
    lib().oracle_sph_density(_d(P), n, _d(r), _d(d), _d(p))
    return d, p


def sph_gradv(q, r, v, d):
    P = sph_params_vector(q)
    r, v, d = _f64(r), _f64(v), _f64(d)
    G = np.zeros((r.shape[0], 4))
    lib().oracle_sph_gradv(_d(P), r.shape[0], _d(r), _d(v), _d(d), _d(G))
    return G.reshape(-1, 2, 2)


def sph_accel(q, r, v, d, p, pi):
    P = sph_params_vector(q)
    r, v, d, p, pi = _f64(r), _f64(v), _f64(d), _f64(p), _f64(pi)
    a = np.zeros((r.shape[0], 2))
    lib().oracle_sph_accel(_d(P), r.shape[0], _d(r), _d(v), _d(d), _d(p), _d(pi), _d(a))
    return a


def sph_step(q, r, v, pi):
    """One macro velocity-Verlet step in place; returns the micro gradients (n, 3, 3)."""
    P = sph_params_vector(q)
    n = r.shape[0]
    d, p, acc, G, L = np.zeros(n), np.zeros(n), np.zeros(2 * n), np.zeros(4 * n), np.zeros(9 * n)
    lib().oracle_sph_step(_d(P), n, _d(r), _d(v), _d(_f64(pi)), _d(d), _d(p), _d(acc), _d(G), _d(L))
    return L.reshape(n, 3, 3)


def sph_polymer_stress(q, sig):
    P = sph_params_vector(q)
    sig = _f64(sig).reshape(-1, 6)
    pi = np.zeros((sig.shape[0], 3))
    lib().oracle_sph_polymer_stress(_d(P), sig.shape[0], _d(sig), _d(pi))
    return pi
