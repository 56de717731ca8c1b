"""Reverse Poiseuille flow to steady state with the coupled LHMM loop
(Sec. "Reverse Poiseuille Flow"; closed forms of Eq. RPF and Appendix
"Analytical velocity profile for pure solvent").

The macro side is set up as the paper does (Lucy kernel of support 4 dh,
Tait pressure with background pressure, exchange interval
delta_t = M_bar dt_SPH = k' dt_micro, see ``inputs.reverse_poiseuille_paper``);
every SPH particle drives one periodic DPD micro-box (solvent plus FENE
chains) under its own velocity gradient, and the boxes' mean stresses come
back as the polymer stress.  After a start-up of several viscous times the
run samples, row by row in y,

* the velocity v_x,
* the solvent shear stress eta_SPH (d_y v_x + d_x v_y) from the SPH
  gradient of Eq. (macro_micro), eta_SPH the shear viscosity the pair
  viscous term of Eq. (sph_continuity) realises (see sph_shear_viscosity),
* the polymer shear stress alpha / lambda* x the micro-domains' sigma_xy,

and compares their sum with the exact steady shear stress of the forcing,
which holds whatever the constitutive behaviour: the momentum balance
d tau_xy / dy = -rho f_x with f_x = -F below mid-height and +F above gives
the triangle wave tau_xy = rho F (y - Ly/4) for y < Ly/2 and
rho F (3 Ly/4 - y) above, of peak rho F Ly / 4.  This is Eq. RPF with the
sign of a tension-positive stress under the stated force directions (the
printed formula carries the opposite sign).  The velocity is compared with
the Newtonian parabola of the total viscosity eta_SPH + eta_p, eta_p the
micro-domains' viscosity measured in the same run (least-squares slope of
the polymer stress against the shear rate).  With n_particles = 0 the run is
the SPH-only Newtonian reference (no micro-domains).

``python -m paper_2512_13267_amd.rpf`` runs the paper's 40 x 40 set-up and
prints a JSON summary (``--md`` writes a report).
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time

import numpy as np

from ._lib import FLAG_BOND, FLAG_CELL, FLAG_NONFINITE, FLAG_THIN


def rpf_shear_stress(y, F: float, rho: float, Ly: float):
    """Exact steady shear stress of the reverse-Poiseuille forcing
    (tension positive; +F x-hat for y >= Ly/2, -F below)."""
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < 0.5 * Ly, rho * F * (y - 0.25 * Ly), rho * F * (0.75 * Ly - y))


def rpf_velocity(y, F: float, rho: float, eta: float, Ly: float):
    """Newtonian steady velocity: a parabola of peak F rho Ly^2 / (32 eta)
    in each half, centred at Ly/4 (flowing along -x) and 3 Ly/4 (+x)."""
    y = np.asarray(y, dtype=np.float64)
    vmax = F * rho * Ly * Ly / (32.0 * eta)
    lower = y < 0.5 * Ly
    yc = np.where(lower, 0.25 * Ly, 0.75 * Ly)
    shape = 1.0 - ((y - yc) / (0.25 * Ly)) ** 2
    return np.where(lower, -vmax, vmax) * shape


def rpf_startup_velocity(y, t: float, F: float, rho: float, eta: float, Ly: float, n_modes: int = 400):
    """Newtonian start-up from rest: v_t = nu v_yy + f(y), nu = eta / rho,
    with the square-wave forcing f = -F (y < Ly/2), +F above, expanded as
    f = -(4F/pi) sum over odd k of sin(2 pi k y / Ly) / k; every mode
    relaxes as (1 - exp(-nu kappa^2 t)) / (nu kappa^2)."""
    y = np.asarray(y, dtype=np.float64)
    nu = eta / rho
    v = np.zeros_like(y)
    for k in range(1, 2 * n_modes, 2):
        kap = 2.0 * math.pi * k / Ly
        lam = nu * kap * kap
        v += -(4.0 * F / math.pi) * np.sin(kap * y) / k * (-math.expm1(-lam * t)) / lam
    return v


def sph_shear_viscosity(eta: float, zeta: float) -> float:
    """Shear viscosity realised by the pair viscous term of Eq.
    (sph_continuity) in 2-D: with friction coefficients a = 2 eta - zeta and
    b = 4 zeta + 2 eta it acts as a/2 + b/8 = 5 eta / 4 (the angular moments
    <e_y^2> = 1/2 and <e_x^2 e_y^2> = 1/8 of the pair direction and
    int F r^2 dA = 2 of a unit-integral kernel).  A b of 4 zeta alone would
    give eta; the coefficients are kept as the paper gives them and the
    factor is accounted for here."""
    a, b = 2.0 * eta - zeta, 4.0 * zeta + 2.0 * eta
    return 0.5 * a + 0.125 * b


def _bin_mean(idx, vals, nb):
    cnt = np.bincount(idx, minlength=nb).astype(np.float64)
    return np.bincount(idx, weights=vals, minlength=nb) / np.maximum(cnt, 1.0)


def run(force: float = 1.0e-2, alpha: float = 0.02, eta_p_guess: float = 0.02, nx: int | None = None,
        n_particles: int = 4000, polymer_fraction: float = 0.1, equil_micro: int = 1000,
        startup: float = 60.0, average: float = 60.0, sample_every: int = 4, n_bins: int = 20,
        replay: int = 10, precision: str = "fp32", micro_model: str = "3d", chain_len: int = 10,
        lam: float | None = None, log=print) -> dict:
    """Coupled reverse-Poiseuille run; startup and average in macro time
    units, replay in exchange intervals.  micro_model "3d": cubic boxes of
    solvent and chains (density 3); "planar": the paper's 2-D melt (Tab. 1,
    n = 4 per unit area, polymer fraction 1, chain_len beads) in planar
    cells, whose 2-D stress (the cell stress times the cell's z edge) is
    what alpha multiplies.  lam: the micro model's relaxation time, for the
    Weissenberg number Wi = 2 U0 lam / L (U0: the mean |v_x|; Sec. "Reverse
    Poiseuille Flow"), with Re = U0 L / (2 eta_tot).  Returns the binned
    profiles and the comparison figures; "flagged_boxes" counts
    box-intervals that ended with a hard flag (cell below 3 rc, bond at R0,
    non-finite stress), "restored_boxes" the box-intervals that were
    restored and replayed."""
    import torch

    from . import inputs, lhmm, micro

    planar = micro_model == "planar"
    if micro_model not in ("3d", "planar"):
        raise ValueError("micro_model must be '3d' or 'planar'")
    mac = inputs.reverse_poiseuille_paper(force=force, alpha=alpha, eta_p=eta_p_guess, nx=nx)
    q = mac.params
    # alpha multiplies the micro-domain's stress in the material's own
    # dimension: for planar cells the engine's (volume) stress times the z edge
    alpha_feed = alpha * (inputs.PLANAR_THICKNESS if planar else 1.0)
    q["alpha"] = alpha_feed
    # planar cells carry no zz stress: their deviatoric part is taken in the plane
    q["micro_dim"] = 2 if planar else 3
    m_bar, k_micro = int(q["m_bar"]), int(q["k_micro"])
    delta_t = m_bar * q["dt"]
    dt_micro = delta_t / k_micro
    coupled = n_particles > 0
    t0 = time.perf_counter()
    sph = lhmm.Sph(q, mac.r, mac.v)
    if coupled:
        if planar:
            wl = inputs.lhmm_boxes(mac.n, n_particles=n_particles, density=4.0, polymer_fraction=1.0, seed_k=21,
                                   planar=True, chain_len=chain_len, dt=dt_micro)
        else:
            wl = inputs.lhmm_boxes(mac.n, n_particles=n_particles, polymer_fraction=polymer_fraction, seed_k=21,
                                   dt=dt_micro)
        mi = micro.from_workload(wl, precision=precision)
        zero = torch.zeros((mac.n, 9), dtype=torch.float64, device="cuda")
        mi.step(zero, equil_micro)
        mi.snapshot()  # the equilibrated state boxes return to when their cell grows thin
        cp = lhmm.Coupled(sph, mi)
        history = collections.deque(maxlen=max(0, int(replay)))
    else:
        L_dev = torch.zeros((mac.n, 9), dtype=torch.float64, device="cuda")
    n_start = int(math.ceil(startup / delta_t))
    n_avg = int(math.ceil(average / delta_t))
    Ly, lam_star = q["Ly"], q["lambda_star"]
    eta_sph = sph_shear_viscosity(q["eta"], q["zeta"])
    edges = np.linspace(0.0, Ly, n_bins + 1)
    yb = 0.5 * (edges[1:] + edges[:-1])
    # reference profiles are binned from the particles' own positions, so
    # they carry the same bin averaging as the measured ones
    samples = {"v": [], "solvent": [], "polymer": [], "rate": [], "shape": [], "tau_ref": [], "speed": []}
    cell_flags = restored = 0
    vmean_trace = []
    for it in range(n_start + n_avg):
        sample = it % sample_every == sample_every - 1
        if coupled:
            cp.step(k_micro, m_bar=m_bar)
            # A periodic box integrates every fluctuation of the gradient into
            # its shape; boxes whose reduced cell has grown thin go back to the
            # equilibrated snapshot and replay the gradients of the last
            # intervals (the micro-domains of the paper are open and have no
            # such shape).
            sig_h, grad_h = cp.coupling_state()
            history.append(grad_h.reshape(-1, 9))
            fl = mi.flags()
            cell_flags += int(np.count_nonzero(fl & (FLAG_CELL | FLAG_BOND | FLAG_NONFINITE)))
            bad = np.nonzero(fl & (FLAG_THIN | FLAG_CELL))[0]
            if bad.size:
                restored += int(bad.size)
                mi.restore(bad)
                for g in history:
                    mi.step_subset(torch.tensor(g, dtype=torch.float64, device="cuda"), k_micro, bad)
        else:
            for j in range(m_bar):
                sph.step(None, L_dev if sample and j == m_bar - 1 else None)
        if sample:
            r, v, _ = sph.get_state()
            if coupled:
                sig, grad = sig_h, grad_h
            else:
                sig, grad = np.zeros((mac.n, 6)), L_dev.cpu().numpy().reshape(-1, 3, 3)
            idx = np.clip(np.searchsorted(edges, r[:, 1], side="right") - 1, 0, n_bins - 1)
            rate = (grad[:, 0, 1] + grad[:, 1, 0]) / lam_star
            vmean_trace.append((round((it + 1) * delta_t, 6), float(np.mean(np.abs(v[:, 0])))))
            if it >= n_start:
                samples["v"].append(_bin_mean(idx, v[:, 0], n_bins))
                samples["rate"].append(_bin_mean(idx, rate, n_bins))
                samples["solvent"].append(_bin_mean(idx, eta_sph * rate, n_bins))
                samples["polymer"].append(_bin_mean(idx, alpha_feed / lam_star * sig[:, 3], n_bins))
                samples["speed"].append(float(np.mean(np.abs(v[:, 0]))))
                unit = rpf_velocity(r[:, 1], 1.0, 1.0, 1.0, Ly) * 32.0 / (Ly * Ly)
                samples["shape"].append(_bin_mean(idx, unit, n_bins))
                samples["tau_ref"].append(_bin_mean(idx, rpf_shear_stress(r[:, 1], force, q["rho0"], Ly), n_bins))
        if log and (it + 1) % 50 == 0:
            log(f"interval {it + 1}/{n_start + n_avg}  t = {(it + 1) * delta_t:.1f}  "
                f"<|v_x|> = {vmean_trace[-1][1]:.4g}", flush=True)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    if coupled:
        mi.close()
    sph.close()

    U0 = float(np.mean(samples.pop("speed")))
    S = {k: np.asarray(a) for k, a in samples.items()}
    ns = S["v"].shape[0]
    mean = {k: a.mean(axis=0) for k, a in S.items()}
    # standard errors from 4 consecutive blocks of samples (correlated samples)
    nblk = 4
    blk = {k: np.stack([b.mean(axis=0) for b in np.array_split(a, nblk)]) for k, a in S.items()}
    se = {k: b.std(axis=0, ddof=1) / math.sqrt(nblk) for k, b in blk.items()}
    total = mean["solvent"] + mean["polymer"]
    total_se = np.sqrt(((blk["solvent"] + blk["polymer"]).std(axis=0, ddof=1) ** 2) / nblk)
    tau_max = q["rho0"] * force * Ly / 4.0
    tau_ref = mean["tau_ref"]
    # away from the force switches at y = 0 and Ly/2, where the kernel smooths
    # the corner of the triangle wave over its support h
    away = np.minimum.reduce([np.abs(yb), np.abs(yb - 0.5 * Ly), np.abs(yb - Ly)]) > q["h"]
    dev = (total - tau_ref) / tau_max
    # polymer viscosity: least-squares slope of the polymer stress on the rate
    g, tp = mean["rate"], mean["polymer"]
    eta_p = float(np.dot(g, tp) / np.dot(g, g))
    eta_tot = eta_sph + eta_p
    vmax_ref = force * q["rho0"] * Ly * Ly / (32.0 * eta_tot)
    shape = mean["shape"]
    v_ref = vmax_ref * shape
    # peak speed: least-squares amplitude of the measured profile on the shape
    vmax_meas = float(np.dot(mean["v"], shape) / np.dot(shape, shape))
    out = {
        "workload": f"reverse Poiseuille flow, {mac.n} SPH particles ({q['Lx']:.1f} x {Ly:.1f}, dh 0.1, Lucy "
                    f"kernel h = {q['h']:.2f}), " + ((f"one {n_particles}-particle 2-D melt micro-domain of {chain_len}-bead "
                                           f"chains per particle (Tab. 1 parameters, planar cell)" if planar else
                                           f"one {n_particles}-particle DPD micro-box per particle") if coupled
                                          else "SPH only (Newtonian reference)"),
        "force": force, "alpha": alpha, "lambda_star": lam_star, "eta_s": q["eta"], "eta_sph": eta_sph, "c": q["c"],
        "micro_model": micro_model, "chain_len": chain_len if planar else None, "U0": U0,
        "Re": U0 * Ly / (2.0 * eta_tot / q["rho0"]), "Wi": (2.0 * U0 * lam / Ly) if lam else None, "lam": lam,
        "theta": q["theta"],
        "dt_sph": q["dt"], "dt_cfl": q["dt_cfl"], "m_bar": m_bar, "k_micro": k_micro, "dt_micro": dt_micro,
        "delta_t": delta_t, "intervals": n_start + n_avg, "startup_intervals": n_start, "samples": ns,
        "n_particles_total": int(mac.n * n_particles), "seconds": seconds, "flagged_boxes": cell_flags,
        "restored_boxes": restored, "replay": replay,
        "tau_max": tau_max, "y": yb.tolist(), "away_from_switches": away.tolist(),
        "v": mean["v"].tolist(), "v_se": se["v"].tolist(), "v_ref": v_ref.tolist(),
        "solvent": mean["solvent"].tolist(), "polymer": mean["polymer"].tolist(), "total": total.tolist(),
        "total_se": total_se.tolist(), "tau_ref": tau_ref.tolist(), "rate": mean["rate"].tolist(),
        "total_dev_rms": float(np.sqrt(np.mean(dev[away] ** 2))), "total_dev_max": float(np.abs(dev[away]).max()),
        "total_dev_rms_all": float(np.sqrt(np.mean(dev ** 2))),
        "eta_p": eta_p, "beta": eta_p / eta_tot, "vmax": float(vmax_meas), "vmax_newtonian": float(vmax_ref),
        "v_shape_rms": float(np.sqrt(np.mean((mean["v"] / vmax_meas - shape) ** 2))),
        "vmean_trace": vmean_trace,
    }
    return out


def report(res: dict, command: str) -> str:
    """Markdown summary of one run."""
    lines = [
        "# Reverse Poiseuille flow to steady state (coupled LHMM)",
        "",
        f"Command: `{command}`",
        "",
        f"Workload: {res['workload']}.  Body force F = {res['force']:g}, alpha = {res['alpha']:g}, "
        f"lambda* = {res['lambda_star']:g}, eta_s = {res['eta_s']:g} (realised by the SPH viscous term as "
        f"{res['eta_sph']:.4g}), sound speed c = {res['c']:.4g}, "
        f"background pressure factor theta = {res['theta']:g}.",
        f"Exchange interval delta_t = {res['delta_t']:.3g} = {res['m_bar']} x dt_SPH {res['dt_sph']:.3g} "
        f"(CFL bound {res['dt_cfl']:.3g}) = {res['k_micro']} x dt_micro {res['dt_micro']:.3g}; "
        f"{res['intervals']} intervals, averages over the last {res['intervals'] - res['startup_intervals']} "
        f"({res['samples']} samples); {res['n_particles_total']:,} DPD particles in all; wall time "
        f"{res['seconds']:.1f} s.  Box-intervals restored from the equilibrated snapshot and replayed over "
        f"{res['replay']} intervals because their cell grew thin: {res['restored_boxes']}; box-intervals with a "
        f"hard flag: {res['flagged_boxes']}.",
        "",
        f"* total shear stress against the exact profile (Eq. RPF, tension-positive sign): RMS deviation "
        f"{res['total_dev_rms']:.3f} tau_max, largest {res['total_dev_max']:.3f} tau_max, over the bins farther "
        f"than h from the force switches (all bins: RMS {res['total_dev_rms_all']:.3f})",
        f"* polymer viscosity from the micro-domains eta_p = {res['eta_p']:.4g}, polymer fraction "
        f"beta = {res['beta']:.3f}",
        f"* mean speed U0 = {res['U0']:.4g}, Re = U0 L / (2 eta_tot) = {res['Re']:.3g}"
        + (f", Wi = 2 U0 lambda / L = {res['Wi']:.3g} with lambda = {res['lam']:g}" if res.get("Wi") else ""),
        f"* peak velocity {res['vmax']:.4g} against the Newtonian {res['vmax_newtonian']:.4g} of "
        f"eta_SPH + eta_p ({res['vmax'] / res['vmax_newtonian']:.3f}); RMS shape deviation of v/v_max "
        f"{res['v_shape_rms']:.3f}",
        "",
        "| y | v_x | v_x Newtonian | solvent tau | polymer tau | total tau | +- | exact tau |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for k, y in enumerate(res["y"]):
        lines.append(f"| {y:.2f} | {res['v'][k]:.4g} | {res['v_ref'][k]:.4g} | {res['solvent'][k]:.3e} | "
                     f"{res['polymer'][k]:.3e} | {res['total'][k]:.3e} | {res['total_se'][k]:.1e} | "
                     f"{res['tau_ref'][k]:.3e} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--force", type=float, default=1.0e-2)
    ap.add_argument("--alpha", type=float, default=0.02)
    ap.add_argument("--nx", type=int, default=None, help="SPH columns (default: a square box)")
    ap.add_argument("--n-particles", type=int, default=4000, help="DPD particles per micro-box (0: SPH only)")
    ap.add_argument("--eta-p-guess", type=float, default=0.02,
                    help="polymer viscosity assumed for the sound speed and time step")
    ap.add_argument("--micro", default="3d", choices=("3d", "planar"),
                    help="micro model: 3-D boxes of solvent and chains, or the paper's 2-D melt")
    ap.add_argument("--chain-len", type=int, default=8, help="beads per chain of the planar melt")
    ap.add_argument("--lam", type=float, default=None, help="micro relaxation time for Wi")
    ap.add_argument("--startup", type=float, default=60.0)
    ap.add_argument("--average", type=float, default=60.0)
    ap.add_argument("--out", default=None, help="JSON output file")
    ap.add_argument("--md", default=None, help="markdown report file")
    ap.add_argument("--command", default=None, help="command line recorded in the report")
    a = ap.parse_args(argv)
    res = run(force=a.force, alpha=a.alpha, eta_p_guess=a.eta_p_guess, nx=a.nx, n_particles=a.n_particles,
              startup=a.startup, average=a.average, micro_model=a.micro, chain_len=a.chain_len, lam=a.lam)
    summary = {k: res[k] for k in ("workload", "intervals", "seconds", "total_dev_rms", "total_dev_max", "eta_p",
                                   "beta", "vmax", "vmax_newtonian", "v_shape_rms", "flagged_boxes",
                                   "restored_boxes", "U0", "Re", "Wi")}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)
    if a.md:
        cmd = a.command or "python -m paper_2512_13267_amd.rpf " + " ".join(argv if argv is not None else sys.argv[1:])
        with open(a.md, "w") as f:
            f.write(report(res, cmd))


if __name__ == "__main__":
    main()
