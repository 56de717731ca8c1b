"""Seeded synthetic workloads for the micro-DPD path.

This module only draws inputs: initial particle states, box shapes, velocity
gradients.  It holds none of the method's arithmetic and imports neither the
HIP binding nor the oracle; both sides receive identical arrays from here.

Every particle coordinate and velocity it returns is exactly representable
in single precision, so a single-precision device state and a
double-precision reference start from the same numbers.

Workloads (the micro-box parameters are those of the polymer model of the
micro-scale section, with the solvent/chain composition and the 3-D periodic
box of the benchmark workloads):
  * ``single_box``: one cubic box of edge 10 rc at number density 3
    (3000 particles, 30 chains of 10 beads), simple shear at rate 0.1;
  * ``batch``: 256 boxes of edge ~U(8, 16) rc at density 3 (1.5k-12k
    particles), polymer fraction ~U(0.1, 0.3) in 10-bead chains, each with a
    constant in-plane traceless gradient whose entries are ~U(-0.5, 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 0x4C484D4D0000  # per-workload seeds are SEED_BASE + k


def default_params(**over) -> dict:
    """DPD/FENE parameters in reduced units (m = rc = kBT = 1)."""
    p = dict(a=25.0, gamma=4.5, sigma=3.0, kBT=1.0, mass=1.0, rc=1.0, dt=0.01, H=30.0, R0=1.5,
             chain_len=10, seed=SEED_BASE + 0)
    p.update(over)
    return p


@dataclass
class BoxInit:
    """Initial state of one micro-box (float64 arrays holding float32 values)."""
    s: np.ndarray          # N x 3 fractional coordinates in [0, 1)
    c: np.ndarray          # N x 3 peculiar velocities
    h: np.ndarray          # 3 x 3 cell, columns are lattice vectors (r = h s)
    n_chains: int
    L: np.ndarray          # 3 x 3 velocity gradient, u = L r
    edge: float = 0.0
    phi: float = 0.0

    @property
    def N(self) -> int:
        return int(self.s.shape[0])


@dataclass
class Workload:
    name: str
    params: dict
    boxes: List[BoxInit] = field(default_factory=list)
    n_steps: int = 0

    @property
    def n_particles(self) -> int:
        return sum(b.N for b in self.boxes)


def _f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _wrap_f32(s: np.ndarray) -> np.ndarray:
    s = s - np.floor(s)
    s32 = s.astype(np.float32)
    s32[s32 >= np.float32(1.0)] = np.float32(0.0)
    s32[s32 < np.float32(0.0)] = np.float32(0.0)
    return s32.astype(np.float64)


def random_box(rng: np.random.Generator, h: np.ndarray, N: int, n_chains: int, chain_len: int,
               kBT: float = 1.0, mass: float = 1.0, b0: float = 0.9, planar: bool = False) -> tuple:
    """Random positions (chains first, as random walks of step b0), Maxwell
    velocities with the mean removed.  Returns (s, c).  planar: a 2-D
    system in the plane z = 0 of the cell (s_z = 0, c_z = 0, walks in the
    plane); every pair separation and force then has a zero z component,
    so the particles never leave the plane (the cell's z edge must be
    diagonal and at least 3 rc)."""
    h = np.asarray(h, dtype=np.float64).reshape(3, 3)
    hinv = np.linalg.inv(h)
    s = rng.random((N, 3))
    if planar:
        if h[0, 2] != 0.0 or h[1, 2] != 0.0 or h[2, 0] != 0.0 or h[2, 1] != 0.0:
            raise ValueError("a planar box needs a cell whose z edge is orthogonal to the plane")
        s[:, 2] = 0.0
    n_beads = n_chains * chain_len
    if n_beads > N:
        raise ValueError("more chain beads than particles")
    if n_chains > 0:
        # random walks of step b0 from a uniform first bead
        u = rng.normal(size=(n_chains, chain_len - 1, 3))
        if planar:
            u[:, :, 2] = 0.0
        u /= np.linalg.norm(u, axis=2, keepdims=True)
        first = s[0:n_beads:chain_len] @ h.T  # (n_chains, 3)
        walk = first[:, None, :] + np.concatenate([np.zeros((n_chains, 1, 3)), np.cumsum(b0 * u, axis=1)],
                                                  axis=1)
        s[:n_beads] = walk.reshape(n_beads, 3) @ hinv.T
    s = _wrap_f32(s)
    c = rng.normal(scale=math.sqrt(kBT / mass), size=(N, 3))
    if planar:
        c[:, 2] = 0.0
    c -= c.mean(axis=0, keepdims=True)
    return s, _f32(c)


def paper_melt_params(chain_len: int = 8, **over) -> dict:
    """DPD/FENE parameters of the paper's 2-D melts (Tab. 1): kBT = 1,
    a = 25, gamma = 4.5 (sigma = 3), m = 1, rc = 1, H = 50, R0 = 1.5,
    dt = 0.005; number density n = 4 per unit area is the box's, not a
    parameter here."""
    p = default_params(a=25.0, gamma=4.5, sigma=3.0, kBT=1.0, mass=1.0, rc=1.0, dt=0.005, H=50.0, R0=1.5,
                       chain_len=chain_len)
    p.update(over)
    return p


def shear_gradient(rate: float) -> np.ndarray:
    """Simple shear u_x = rate * y."""
    L = np.zeros((3, 3))
    L[0, 1] = rate
    return L


def planar_gradient(a: float, b: float, c: float) -> np.ndarray:
    """In-plane traceless gradient [[a, b, 0], [c, -a, 0], [0, 0, 0]]."""
    return np.array([[a, b, 0.0], [c, -a, 0.0], [0.0, 0.0, 0.0]])


def cubic_cell(edge: float) -> np.ndarray:
    return np.diag([edge, edge, edge]).astype(np.float64)


# ---------------------------------------------------------------------------
# Box shapes that survive a constant hyperbolic gradient
# ---------------------------------------------------------------------------

_ENUM_K = 8


def _enum_coeffs(K: int = _ENUM_K) -> np.ndarray:
    m, n = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    mn = np.stack([m.ravel(), n.ravel()], axis=0).astype(np.float64)
    return mn[:, (mn[0] != 0) | (mn[1] != 0)]


def _lattice_min_widths(B: np.ndarray, K: int = _ENUM_K) -> np.ndarray:
    """Largest achievable minimum perpendicular width of each 2-D lattice in
    the stack B (..., 2, 2) (basis in columns): area / (second successive
    minimum), found by enumerating lattice vectors m b1 + n b2 with
    |m|, |n| <= K."""
    B = np.asarray(B, dtype=np.float64)
    shp = B.shape[:-2]
    B = B.reshape(-1, 2, 2)
    area = np.abs(B[:, 0, 0] * B[:, 1, 1] - B[:, 0, 1] * B[:, 1, 0])
    V = B @ _enum_coeffs(K)  # (n, 2, M)
    lens = np.hypot(V[:, 0], V[:, 1])
    k1 = np.argmin(lens, axis=1)
    v1 = V[np.arange(len(B)), :, k1]  # (n, 2)
    l1 = lens[np.arange(len(B)), k1]
    cross = v1[:, :1] * V[:, 1] - v1[:, 1:] * V[:, 0]
    indep = np.abs(cross) > 1e-9 * l1[:, None] * lens
    l2 = np.where(indep, lens, np.inf).min(axis=1)
    return (area / l2).reshape(shp)


def _lattice_min_width(B: np.ndarray, K: int = _ENUM_K) -> float:
    return float(_lattice_min_widths(np.asarray(B)[None], K)[0])


def _flow_maps(L2: np.ndarray, ts: np.ndarray) -> np.ndarray:
    from scipy.linalg import expm
    return expm(np.asarray(L2)[None] * np.asarray(ts)[:, None, None])


def _flow_map(L2: np.ndarray, t: float) -> np.ndarray:
    return _flow_maps(L2, np.array([t]))[0]


def _min_width_over(L2: np.ndarray, B: np.ndarray, t_end: float, samples: int) -> float:
    E = _flow_maps(L2, np.linspace(0.0, t_end, samples))
    return float(_lattice_min_widths(E @ B).min())


def kr_cell(L: np.ndarray, edge: float, t_run: float, min_width: float = 3.5,
            ratios: Optional[np.ndarray] = None) -> tuple:
    """Initial in-plane lattice for a constant in-plane gradient L.

    Returns (h0, kind) with kind "cubic", "kr" or "rotated".  A cubic cell is
    kept when its reduced lattice stays at least ``min_width`` wide over
    ``t_run``; a rotational or shear-like gradient (a^2 + bc <= 0) otherwise
    gets the best rotated square lattice.
    Otherwise, for a hyperbolic L (a^2 + bc > 0), the lattice is aligned in
    the manner of Kraynik and Reinelt: its basis P satisfies
    exp(L T) P = P M with M = [[2, 1], [1, 1]], so the flow maps the lattice
    onto itself every period T = ln(mu)/k, mu = (3 + sqrt 5)/2.  Among the
    one-parameter family P = V diag(d1, d2) W^-1 (V, W eigenvectors of L and
    M) of area edge^2, the member whose minimum width over one period is
    largest is chosen; the returned basis is the lattice's reduced one.  The
    z extent stays ``edge``."""
    L2 = np.asarray(L, dtype=np.float64)[:2, :2]
    cube = np.eye(2) * edge
    if _min_width_over(L2, cube, t_run, 61) >= min_width:
        return cubic_cell(edge), "cubic"
    a, b, c = L2[0, 0], L2[0, 1], L2[1, 0]
    k2 = a * a + b * c
    if k2 <= 0.0:
        return _rotated_square_cell(L2, edge, t_run), "rotated"
    k = math.sqrt(k2)
    evals, V = np.linalg.eig(L2)
    V = np.real(V[:, np.argsort(-np.real(evals))])  # columns: +k, -k
    mu = (3.0 + math.sqrt(5.0)) / 2.0
    W = np.array([[1.0, 1.0], [mu - 2.0, 1.0 / mu - 2.0]])  # eigenvectors of M for mu, 1/mu
    Winv = np.linalg.inv(W)
    T = math.log(mu) / k
    if ratios is None:
        ratios = np.exp(np.linspace(-4.0, 4.0, 81))
    E = _flow_maps(L2, np.linspace(0.0, T, 25))  # (25, 2, 2)
    cands = []
    for sgn in (1.0, -1.0):
        for r in ratios:
            P = V @ np.diag([r, sgn]) @ Winv
            det = np.linalg.det(P)
            if abs(det) < 1e-300:
                continue
            P = P * math.sqrt(edge * edge / abs(det))
            if np.linalg.det(P) < 0:
                P = P[:, ::-1].copy()
            cands.append(P)
    cands = np.stack(cands)  # (C, 2, 2)
    widths = _lattice_min_widths(E[:, None] @ cands[None]).min(axis=0)  # (C,)
    bestP = cands[int(np.argmax(widths))]
    M = np.linalg.inv(bestP) @ _flow_map(L2, T) @ bestP
    assert np.allclose(M, np.round(M), atol=1e-6)
    h = np.zeros((3, 3))
    h[:2, :2] = _short_basis(bestP)
    h[2, 2] = edge
    return h, "kr"


def _rotated_square_cell(L2: np.ndarray, edge: float, t_run: float, angles: int = 46) -> np.ndarray:
    """For a rotational or shear-like (a^2 + bc <= 0) gradient whose cubic
    cell narrows: the square lattice of side ``edge`` rotated to the angle
    whose minimum width over ``t_run`` is largest (these flows stretch a
    lattice at most linearly in time, so a wide enumeration suffices)."""
    E = _flow_maps(L2, np.linspace(0.0, t_run, 81))
    best, bestB = -1.0, None
    for th in np.linspace(0.0, 0.5 * math.pi, angles, endpoint=False):
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]) * edge
        w = float(_lattice_min_widths(E @ R, K=24).min())
        if w > best:
            best, bestB = w, R
    h = np.zeros((3, 3))
    h[:2, :2] = _short_basis(bestB)
    h[2, 2] = edge
    return h


def _short_basis(B: np.ndarray, K: int = 12) -> np.ndarray:
    """The lattice's two successive minima (a reduced basis of the same 2-D
    lattice), oriented with positive determinant."""
    m, n = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    m = m.ravel()
    n = n.ravel()
    keep = (m != 0) | (n != 0)
    m, n = m[keep], n[keep]
    V = np.outer(B[:, 0], m) + np.outer(B[:, 1], n)
    lens = np.hypot(V[0], V[1])
    order = np.argsort(lens, kind="stable")
    v1 = V[:, order[0]]
    for k in order[1:]:
        v2 = V[:, k]
        cross = v1[0] * v2[1] - v1[1] * v2[0]
        if abs(cross) > 1e-9 * lens[order[0]] * lens[k]:
            if cross < 0:
                v2 = -v2
            out = np.stack([v1, v2], axis=1)
            assert abs(abs(np.linalg.det(out)) - abs(np.linalg.det(B))) < 1e-9 * abs(np.linalg.det(B))
            return out
    raise ValueError("degenerate lattice")


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_box(seed_k: int = 0, edge: float = 10.0, density: float = 3.0, polymer_fraction: float = 0.1,
               shear_rate: float = 0.1, n_steps: int = 500, **param_over) -> Workload:
    """One cubic box in simple shear (3000 particles, 30 chains at edge 10)."""
    p = default_params(seed=SEED_BASE + seed_k, **param_over)
    rng = np.random.default_rng(SEED_BASE + seed_k)
    N = int(round(density * edge ** 3))
    n_chains = int(round(polymer_fraction * N / p["chain_len"]))
    h = cubic_cell(edge)
    s, c = random_box(rng, h, N, n_chains, p["chain_len"], p["kBT"], p["mass"])
    box = BoxInit(s=s, c=c, h=h, n_chains=n_chains, L=shear_gradient(shear_rate), edge=edge,
                  phi=polymer_fraction)
    return Workload("single_box", p, [box], n_steps)


def batch(n_boxes: int = 256, seed_k: int = 1, edge_range=(8.0, 16.0), density: float = 3.0,
          phi_range=(0.1, 0.3), grad_range: float = 0.5, n_steps: int = 2000, kr: bool = True,
          **param_over) -> Workload:
    """Boxes of uneven size, each under its own constant in-plane gradient."""
    p = default_params(seed=SEED_BASE + seed_k, **param_over)
    rng = np.random.default_rng(SEED_BASE + seed_k)
    boxes = []
    t_run = n_steps * p["dt"]
    for _ in range(n_boxes):
        edge = float(rng.uniform(*edge_range))
        N = int(round(density * edge ** 3))
        phi = float(rng.uniform(*phi_range))
        n_chains = int(round(phi * N / p["chain_len"]))
        a, b, c = rng.uniform(-grad_range, grad_range, size=3)
        L = planar_gradient(a, b, c)
        if kr:
            h, _ = kr_cell(L, edge, t_run)
        else:
            h = cubic_cell(edge)
        s, cc = random_box(rng, h, N, n_chains, p["chain_len"], p["kBT"], p["mass"])
        boxes.append(BoxInit(s=s, c=cc, h=h, n_chains=n_chains, L=L, edge=edge, phi=phi))
    return Workload("batch", p, boxes, n_steps)


def tiny_boxes(n_boxes: int, seed_k: int = 7, edges=(4.2, 5.0, 6.3), density: float = 3.0,
               phi: float = 0.2, grad_scale: float = 0.3, **param_over) -> Workload:
    """Small ragged boxes for parity tests (sizes cycle through ``edges``)."""
    p = default_params(seed=SEED_BASE + seed_k, **param_over)
    rng = np.random.default_rng(SEED_BASE + seed_k)
    boxes = []
    for b in range(n_boxes):
        edge = float(edges[b % len(edges)])
        N = int(round(density * edge ** 3))
        n_chains = int(round(phi * N / p["chain_len"]))
        a, bb, c = rng.uniform(-grad_scale, grad_scale, size=3)
        L = planar_gradient(a, bb, c)
        h = cubic_cell(edge)
        s, cc = random_box(rng, h, N, n_chains, p["chain_len"], p["kBT"], p["mass"])
        boxes.append(BoxInit(s=s, c=cc, h=h, n_chains=n_chains, L=L, edge=edge, phi=phi))
    return Workload("tiny_boxes", p, boxes, 0)


# ---------------------------------------------------------------------------
# Macro (SPH) workloads
# ---------------------------------------------------------------------------

@dataclass
class MacroInit:
    """Initial SPH state and parameters of a 2-D periodic macro problem."""
    r: np.ndarray           # n x 2 positions
    v: np.ndarray           # n x 2 velocities
    params: dict
    n_steps: int = 0

    @property
    def n(self) -> int:
        return int(self.r.shape[0])


KERNELS = {"quintic": 0, "lucy": 1}
SUPPORT = {"quintic": 3.0, "lucy": 4.0}   # support radius h in units of the spacing dh


def sound_speed(v_max: float, eta_tot: float, length: float, f_ext: float, delta: float = 0.1) -> float:
    """Artificial sound speed, Eq. (sound_speed) (Appendix "Artificial sound
    speed"): the largest of v_max/delta, sqrt(eta_tot v_max / (delta L)) and
    sqrt(|f| L / delta), so that the Mach number stays near delta."""
    return max(v_max / delta, math.sqrt(eta_tot * v_max / (delta * length)), math.sqrt(abs(f_ext) * length / delta))


def cfl_dt(h: float, v_max: float, c: float, f_ext: float, nu: float, safety: float = 0.25) -> float:
    """SPH time step of Eq. (cfl_condition): safety x the smallest of the
    acoustic limit h/(|v|max + c), the body-force limit (h/|f|)^(1/2) and
    the viscous limit h^2/(2 nu); a zero force or viscosity drops its limit."""
    lims = [h / (v_max + c)]
    if f_ext != 0.0:
        lims.append(math.sqrt(h / abs(f_ext)))
    if nu > 0.0:
        lims.append(h * h / (2.0 * nu))
    return safety * min(lims)


def reverse_poiseuille(nx: int = 16, ny: int = 64, width: float = 1.0, force: float = 0.2, eta_s: float = 0.1,
                       beta: float = 0.5, rho0: float = 1.0, dt: float = 1e-3, lambda_star: float = 0.2,
                       alpha: float = 0.07, theta: float = 0.5, n_steps: int = 200,
                       kernel: str = "quintic") -> MacroInit:
    """Reverse Poiseuille flow: a periodic channel of two counter-flowing
    halves of the given width (Ly = 2 width), body force +force along x for
    y >= width and -force below, SPH particles on an nx x ny lattice of
    spacing dh = 2 width / ny; quintic kernel of support h = 3 dh, or the
    Lucy kernel of support h = 4 dh (kernel="lucy").  The sound speed
    follows Eq. (sound_speed) with delta = 0.1, the characteristic length =
    width and the expected peak velocity of the Newtonian profile
    force width^2 / (8 nu_tot), nu_tot = eta_s / ((1 - beta) rho0)."""
    dh = 2.0 * width / ny
    Lx, Ly = nx * dh, ny * dh
    eta_tot = eta_s / (1.0 - beta)
    vmax = force * width * width / (8.0 * eta_tot / rho0)
    c = sound_speed(vmax, eta_tot, width, force)
    xs, ys = np.meshgrid((np.arange(nx) + 0.5) * dh, (np.arange(ny) + 0.5) * dh, indexing="ij")
    r = np.stack([xs.ravel(), ys.ravel()], axis=1)
    params = dict(rho0=rho0, eta=eta_s, zeta=0.0, c=c, theta=theta, F=force, h=SUPPORT[kernel] * dh, dt=dt,
                  mass=rho0 * dh * dh, Lx=Lx, Ly=Ly, lambda_star=lambda_star, alpha=alpha, n_fixed=0, force_mode=0,
                  kernel=KERNELS[kernel])
    return MacroInit(r=r, v=np.zeros_like(r), params=params, n_steps=n_steps)


def reverse_poiseuille_paper(force: float = 1.0e-2, eta_s: float = 0.02, eta_p: float = 0.02, L: float = 4.0,
                             nx: int | None = None, dh: float = 0.1, rho0: float = 1.0, lambda_star: float = 1.0,
                             alpha: float = 0.02, theta: float = 0.5, delta_t: float = 0.32,
                             dt_sph: float | None = 0.04, dt_micro: float = 0.005) -> MacroInit:
    """Reverse Poiseuille flow set up as in the paper (Sec. "Reverse
    Poiseuille Flow"): a periodic box of height Ly = L = 4 (and width L, or
    nx columns), SPH spacing dh = 0.1, rho = 1, solvent viscosity 0.02, the
    Lucy kernel of support h = 4 dh and the Tait equation with background
    pressure theta c^2 rho0 / 7.  The sound speed follows Eq. (sound_speed)
    with the Newtonian peak velocity of Appendix "Analytical velocity
    profile", force rho0 L^2 / (32 eta_tot), eta_tot = eta_s + eta_p (eta_p:
    the viscosity the micro-domains are expected to add).  The exchange
    interval is delta_t = M_bar dt_SPH = k' dt_micro (Sec. "Temporal Coupling
    Scheme"; the paper: 0.32 = 8 x 0.04 = 64 x 0.005).  dt_SPH is the given
    step (None: the step of Eq. (cfl_condition)), lowered if needed so that
    it stays within Eq. (cfl_condition) and M_bar = delta_t / dt_SPH is an
    integer.  params carries "m_bar", "k_micro", "dt_cfl", "eta_tot" and
    "v_max" beside the engine parameters."""
    n_y = int(round(L / dh))
    n_x = n_y if nx is None else int(nx)
    eta_tot = eta_s + eta_p
    vmax = force * rho0 * L * L / (32.0 * eta_tot)
    c = sound_speed(vmax, eta_tot, L, force)
    h = SUPPORT["lucy"] * dh
    dt_cfl = cfl_dt(h, vmax, c, force, eta_tot / rho0)
    dt = dt_cfl if dt_sph is None else min(float(dt_sph), dt_cfl)
    m_bar = max(1, int(math.ceil(delta_t / dt - 1e-9)))
    k_micro = int(round(delta_t / dt_micro))
    xs, ys = np.meshgrid((np.arange(n_x) + 0.5) * dh, (np.arange(n_y) + 0.5) * dh, indexing="ij")
    r = np.stack([xs.ravel(), ys.ravel()], axis=1)
    params = dict(rho0=rho0, eta=eta_s, zeta=0.0, c=c, theta=theta, F=force, h=h, dt=delta_t / m_bar,
                  mass=rho0 * dh * dh, Lx=n_x * dh, Ly=n_y * dh, lambda_star=lambda_star, alpha=alpha, n_fixed=0,
                  force_mode=0, kernel=KERNELS["lucy"], m_bar=m_bar, k_micro=k_micro, dt_cfl=dt_cfl,
                  eta_tot=eta_tot, v_max=vmax)
    return MacroInit(r=r, v=np.zeros_like(r), params=params)


def cylinder_array(n: int = 64, radius: float = 0.2, force: float = 1.0, eta_s: float = 0.1, beta: float = 0.5,
                   rho0: float = 1.0, dt: float = 1e-3, lambda_star: float = 0.2, alpha: float = 0.07,
                   theta: float = 0.5, n_steps: int = 500) -> MacroInit:
    """Flow past a periodic square array of cylinders: the unit cell [0, 1)^2
    with one cylinder of the given radius at its centre, SPH particles on an
    n x n lattice of spacing dh = 1/n (support h = 3 dh); lattice sites inside
    the cylinder become frozen wall particles, stored after the fluid ones
    (params["n_fixed"] of them).  A uniform body force +force x-hat drives
    the flow (params["force_mode"] = 1).  The sound speed follows
    Eq. (sound_speed) with delta = 0.1 and the radius as length scale."""
    dh = 1.0 / n
    xs, ys = np.meshgrid((np.arange(n) + 0.5) * dh, (np.arange(n) + 0.5) * dh, indexing="ij")
    r = np.stack([xs.ravel(), ys.ravel()], axis=1)
    inside = np.hypot(r[:, 0] - 0.5, r[:, 1] - 0.5) < radius
    r = np.concatenate([r[~inside], r[inside]])
    eta_tot = eta_s / (1.0 - beta)
    gap = 1.0 - 2.0 * radius
    vmax = force * gap * gap / (8.0 * eta_tot / rho0)
    c = sound_speed(vmax, eta_tot, radius, force)
    params = dict(rho0=rho0, eta=eta_s, zeta=0.0, c=c, theta=theta, F=force, h=3.0 * dh, dt=dt,
                  mass=rho0 * dh * dh, Lx=1.0, Ly=1.0, lambda_star=lambda_star, alpha=alpha,
                  n_fixed=int(inside.sum()), force_mode=1)
    return MacroInit(r=r, v=np.zeros_like(r), params=params, n_steps=n_steps)


PLANAR_THICKNESS = 3.5  # z edge of a planar cell: above the 3.3 rc at which a cell counts as thin


def lhmm_boxes(n_boxes: int, n_particles: int = 4000, density: float = 3.0, polymer_fraction=0.1,
               seed_k: int = 2, planar: bool = False, **param_over) -> Workload:
    """One cubic micro-box per SPH particle, each of n_particles at the given
    density (edge (n/density)^(1/3)), chains holding the polymer fraction (a
    number, or one value per box), random start, no gradient (the macro side
    supplies it).  planar: the paper's 2-D material instead (Tab. 1
    parameters unless overridden, density per unit area, edge
    (n/density)^(1/2)), held in the plane z = 0 of a cell of z edge
    PLANAR_THICKNESS; its 2-D stress is the cell stress times that edge."""
    if planar:
        p = paper_melt_params(seed=SEED_BASE + seed_k, **param_over)
        edge = (n_particles / density) ** 0.5
        h = np.diag([edge, edge, PLANAR_THICKNESS])
    else:
        p = default_params(seed=SEED_BASE + seed_k, **param_over)
        edge = (n_particles / density) ** (1.0 / 3.0)
        h = cubic_cell(edge)
    rng = np.random.default_rng(SEED_BASE + seed_k)
    phis = np.broadcast_to(np.asarray(polymer_fraction, dtype=np.float64), (n_boxes,))
    boxes = []
    for b in range(n_boxes):
        n_chains = int(phis[b] * n_particles) // p["chain_len"] if planar else \
            int(round(phis[b] * n_particles / p["chain_len"]))
        s, c = random_box(rng, h, n_particles, n_chains, p["chain_len"], p["kBT"], p["mass"], planar=planar)
        boxes.append(BoxInit(s=s, c=c, h=h, n_chains=n_chains, L=np.zeros((3, 3)), edge=edge, phi=float(phis[b])))
    return Workload("lhmm_boxes", p, boxes, 0)
